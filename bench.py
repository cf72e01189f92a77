"""Benchmark: batched Hirsch-Fye QMC proposals/s on one MI355X.

Workload (the spec configuration): 512 impurities at L = 64
(beta = 8, dtau = 0.125), U ~ U[4, 12], Weiss functions of the centre site of
an open 64-site chain at mu_eff ~ U[-1, 1] (seed 3), 200 warm-up + 2000
measured sweeps each, fp64, Dyson recompute every 50 sweeps, 32 bins.

A step is one pass of the whole hot path over the batch: field
initialisation, from-scratch Dyson, all sweeps with Sherman-Morrison updates,
periodic recomputes, measurement and binning -- one hfqmc_run on inputs
already resident in HBM, followed by a stream synchronisation.

Prints ONE JSON line (rank 0).  `value` is proposals/s of the whole job;
`roofline` prices the sweep kernel's algorithmic fp64 flops against the
MI355X fp64 vector peak; `cpu_baseline` times the CPU oracle on a bounded
sample of the same workload on the host cores.

Other workloads (one JSON line each, --workload NAME or all):
  uneven   512 impurities, L ~ U{32,48,64,96,128}, beta = 8: untuned vs
           autotuned fp64, and fp32 flush products (window and delayed k = 16)
           under the drift limit, with refused impurities, drift and g(tau)
           shift against the fp64 path
  long     128 impurities at L = 160 (G in device memory): window updates vs
           delayed updates (k = 16), time per proposal of a chain
  serving  Poisson request stream (200/s), L in {20,40,80,160} (4:3:2:1),
           U = 8, dtau = 0.25, 5000 sweeps, 200 sites x 10 DMFT iterations
           with device-resident state: p50/p99 latency and throughput;
           --serve-chains N splits each L = 160 request into N chains
           (serving_chains: the same stream with 4 chains per L = 160 request)
  trapped  21x21 trap (V0 = 0.05, U = 8, beta = 10, L = 40, AF seed), the
           325 sites with n > 1e-3, 1000 + 10000 sweeps, fp64
  slab     41x41 trap (V0 = 0.02, U = 8, beta = 16, L = 80, ~1000 atoms,
           AF seed), 1281 sites, 1000 + 10000 sweeps; fp64 and fp32 flush
           products under the drift limit (refused sites counted)
  rdmft    one real-space DMFT iteration of the 21x21 trap: lattice Green
           function at 500 Matsubara frequencies, Weiss functions, the
           325-site solve, self-energy; the lattice part alone on 41x41
  trotter  dtau -> 0: the 21x21 trap's sites at L = 32, 40, 50 in one batch,
           fitted even in dtau
  thermo   entropy from dS/dmu = dN/dT: 13x13 trap, U = 10, converged RDMFT
           at 45 chemical potentials x 2 temperatures
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6  # 256 CU x 2.4 GHz x 128 fp64 flop/clk/CU (fp64 MFMA: the same)
FP32_MFMA_PEAK_TFLOPS = 157.3
RECOMPUTE_EVERY = 50

# HBM bytes per launch of the dominant kernel on this workload, from
# rocprofv3 FETCH_SIZE/WRITE_SIZE scaled by a 256 MiB copy (profiles/),
# valid only for the kernel sources with the sha256 prefix recorded with them.
PROFILED_TRAFFIC = {
    # kernel: (source files, sha256 prefix, bytes per launch)
    "hfqmc::sweep_kernel<Cfg<64,2,0>>": (("hfqmc_sweep.hip", "hfqmc_device.h", "hfqmc_internal.h"),
                                         "17d1141ae7a6dc7b", 2.5545e7),
}


# lattice Green function kernel (21 x 21 trap, 500 frequencies x 2 spins):
# FETCH_SIZE x 1.9997 + WRITE_SIZE of one launch, almost all of it the
# workspace round trip of the left-connected inverses
PROFILED_LATTICE_SHA = "8bb37110995ab5b7"
PROFILED_LATTICE_TRAFFIC_BYTES = 6.866e8


def kernel_sha(files=("hfqmc_sweep.hip", "hfqmc_device.h", "hfqmc_internal.h")) -> str:
    """sha256 prefix of a kernel's sources (default: the register-tile sweep kernel)."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1006_2716_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def kernel_traffic(kernel: str):
    ent = PROFILED_TRAFFIC.get(kernel)
    if ent is None:
        return None
    files, sha, traffic = ent
    return traffic if kernel_sha(files) == sha else None


def lattice_traffic():
    same = kernel_sha(("hfqmc_lattice.hip", "hfqmc_lattice.h")) == PROFILED_LATTICE_SHA
    return PROFILED_LATTICE_TRAFFIC_BYTES if same else None


def algorithmic_flops(L: int, p_acc: float, n_rec: int = RECOMPUTE_EVERY, kbar: float = 0.0) -> float:
    """Flops per proposal, both spins, FMA = 2 flops: rank-one (or flush)
    4 p L^2, delayed column/row 8 p L kbar, Dyson (16/3) L^2 / n_rec,
    measurement 2 L."""
    return 4.0 * p_acc * L * L + 8.0 * p_acc * L * kbar + (16.0 / 3.0) * L * L / n_rec + 2.0 * L


def host_cpu():
    """CPU model (from /proc/cpuinfo), logical CPUs of the host, CPUs this
    process may run on, and the threads the oracle uses: the host-core share
    this process is given (OMP_NUM_THREADS when set), else every CPU of its
    affinity mask."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    affinity = len(os.sched_getaffinity(0))
    share = os.environ.get("OMP_NUM_THREADS", "")
    threads = int(share) if share.isdigit() and int(share) > 0 else affinity
    return dict(model=model, nproc=os.cpu_count() or 1, affinity=affinity, threads=min(threads, affinity))


def cpu_baseline(probs, seconds_hint: float = 12.0, chunk: int = 128):
    """The oracle on the host's cores: impurities of the step in order, a
    chunk at a time (at least one), until the whole step is done or
    seconds_hint has passed (a bounded sample on a slow host)."""
    import oracle
    cpu = host_cpu()
    threads = cpu["threads"]
    done, props = 0, 0
    t0 = time.perf_counter()
    while done < len(probs) and (done == 0 or time.perf_counter() - t0 < seconds_hint):
        res = oracle.run(probs[done:done + chunk], n_threads=threads)
        props += sum(r["proposals"] for r in res)
        done += len(res)
    dt = time.perf_counter() - t0
    what = "all" if done == len(probs) else f"first {done} of"
    return dict(value=props / dt, unit="proposals/s", cores=threads, kind="oracle",
                per_core=props / dt / threads, cpu_model=cpu["model"], host_nproc=cpu["nproc"],
                affinity_cpus=cpu["affinity"],
                threads_rule="OMP_NUM_THREADS (this process's host-core share) if set, else the affinity mask",
                sample=f"{what} {len(probs)} impurities in chunks of {chunk}, full {probs[0]['n_warmup']}+"
                       f"{probs[0]['n_measure']} sweeps ({props} proposals, {dt:.1f} s)")


def single_impurity_rate(ctx, probs, n: int = 8):
    """The plain single-impurity GPU path: one impurity per launch, in turn."""
    import torch
    total, t_all = 0, 0.0
    for p in probs[:n]:
        ctx.stage([p])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.run()
        torch.cuda.synchronize()
        t_all += time.perf_counter() - t0
        total += (p["n_warmup"] + p["n_measure"]) * p["L"]
    return total / t_all


def timed_runs(ctx, steps, warmup, graph=False):
    """Run the staged batch; returns (wall ms per step, per-step ms list,
    per-step kernel ms of launch 0 or of the whole pass)."""
    import torch
    run = ctx.run_graph if graph else ctx.run
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    step_ms, kern_ms = [], []
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - t0) * 1e3)
        kern_ms.append(ctx.last_run_ms()[0] if graph else ctx.last_launch_ms(0)[0])
    torch.cuda.synchronize()
    return (time.perf_counter() - t_start) * 1e3 / steps, step_ms, kern_ms


def _line(metric, value, unit, steps, warmup, ms, config, dtype="f64", **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def _g_shift(a, b):
    """max |g_a - g_b| and max |g_a - g_b| / sigma_comb over tau, spins, impurities."""
    dmax, zmax = 0.0, 0.0
    for x, y in zip(a, b):
        for s in ("up", "dn"):
            d = np.abs(x[f"g_{s}"] - y[f"g_{s}"])
            e = np.sqrt(x[f"g_{s}_err"] ** 2 + y[f"g_{s}_err"] ** 2)
            dmax = max(dmax, float(d.max()))
            zmax = max(zmax, float((d[e > 0] / e[e > 0]).max()))
    return dmax, zmax


def bench_uneven(args):
    import torch
    from paper_1006_2716_amd import hfqmc, workloads
    probs = workloads.chain_batch(n_imp=512, Ls=(32, 48, 64, 96, 128), seed=3)
    props = sum((p["n_warmup"] + p["n_measure"]) * p["L"] for p in probs)
    ctx = hfqmc.Context(0)
    ws = ctx.alloc_workspace(probs)
    ctx.stage(probs, ws)
    ms_def, _, _ = timed_runs(ctx, args.steps, args.warmup)
    ref = ctx.collect()
    t0 = time.perf_counter()
    ctx.tune(probs, sweeps=64, workspace=ws)
    tune_s = time.perf_counter() - t0
    plans = {L: ctx.plan(L, 0)[:2] for L in (32, 48, 64, 96, 128)}
    ctx.stage(probs, ws)
    ms_tuned, step_ms, _ = timed_runs(ctx, args.steps, args.warmup)
    launches = [ctx.last_launch_ms(i) for i in range(ctx.last_run_ms()[1])]
    # fp32 flush products (window updates, the precision's default, and
    # delayed k = 16) under the context's drift limit: impurities whose drift
    # the limit cannot hold end HFQMC_ENUMERIC and are counted, not used
    mixed = {}
    mctx = hfqmc.Context(0, precision=hfqmc.MIXED)
    for k in (0, 16):
        pk = [dict(p, delay=k) for p in probs]
        mctx.stage(pk, ws)
        ms_k, _, _ = timed_runs(mctx, 1, 0)
        rk = mctx.collect()
        ok = [i for i, x in enumerate(rk) if x["status"] == 0]
        dmax, zmax = _g_shift([rk[i] for i in ok], [ref[i] for i in ok])
        mixed["window" if k == 0 else f"delayed_k{k}"] = dict(
            proposals_per_s=props / (ms_k * 1e-3), ms=ms_k, failed=len(rk) - len(ok),
            max_drift=max(rk[i]["max_drift"] for i in ok), max_g_shift_vs_fp64=dmax, max_g_shift_sigma=zmax)
    torch.cuda.synchronize()
    _line("HF-QMC spin-flip proposals/s (batched impurities, uneven L)", props / (ms_tuned * 1e-3), "proposals/s",
          args.steps, args.warmup, ms_tuned,
          {"workload": "512 impurities, L~U{32,48,64,96,128}, beta=8, U~U[4,12], open 64-site chain centre-site "
                       "Weiss at mu_eff~U[-1,1] (seed 3), 200+2000 sweeps, fp64, autotuned shapes",
           "proposals_per_step": props, "untuned_proposals_per_s": props / (ms_def * 1e-3),
           "tune_seconds": round(tune_s, 2), "plan_rt_k_by_L": {str(L): v for L, v in plans.items()},
           "class_launch_ms_L_items": launches},
          p99_solve_ms=float(np.percentile(step_ms, 99)), mixed_fp32_products=mixed)
    mctx.close()
    ctx.close()


def bench_serving(args):
    from paper_1006_2716_amd import hfqmc, serve_load, workloads
    sites, arrivals, weiss = workloads.serving_requests()
    for s in sites:  # the device-memory kernel class bounds the tail: split it into chains
        if s["L"] > 128 and args.serve_chains > 1:
            s["n_chains"] = args.serve_chains
    ctx = hfqmc.Context(0, tune_cache=args.tune_cache)
    ctx.attach_pool(1 << 30)
    ctx.serve_config(step_ms=args.step_ms, quantum_proposals=args.quantum)
    t0 = time.perf_counter()
    out = serve_load.replay(ctx, sites, arrivals, weiss, n_iter=10, sweeps=5000, warm_first=500, warm_next=100,
                            progress=lambda m: print(m, file=sys.stderr, flush=True))
    wall = time.perf_counter() - t0
    st = ctx.serve_stats()
    ctx.close()
    out.pop("results")
    name = "HF-QMC serving: p99 request latency (Poisson 200 req/s)"
    if args.serve_chains > 1:
        name += f", L = 160 requests as {args.serve_chains} chains"
    _line(name, out["p99_ms"], "ms", 1, 0, wall * 1e3,
          {"workload": "Poisson 200 req/s, L in {20,40,80,160} weights 4:3:2:1, U=8, dtau=0.25, 5000 sweeps "
                       "(500 warm-up first, 100 later), 200 sites x 10 DMFT iterations, state on device",
           "step_ms": args.step_ms, "quantum_proposals": args.quantum, "chains_L160": max(1, args.serve_chains),
           "steps": st["steps"],
           "launches": st["launches"], "step_ms_avg": st["step_ms_avg"], "launch_ms_avg": st["launch_ms_avg"]},
          higher_is_better=False, serving=out)


def bench_long(args):
    """L = 160 (G in device memory): 128 requests of the serving generator
    (U = 8, dtau = 0.25) as one batch, window updates (the default) and
    delayed updates (k = 16); time per proposal of one chain."""
    from paper_1006_2716_amd import hfqmc, workloads
    sites, _, weiss = workloads.serving_requests(n_sites=512, Ls=(160,), weights=(1,), seed=4)
    probs = [dict(L=160, beta=s["beta"], U=s["U"], weiss=weiss(s, 0), n_warmup=200, n_measure=2000, recompute_every=50,
                  n_bins=32, seed=s["seed"], site=s["site"]) for s in sites[:128]]
    props = sum((p["n_warmup"] + p["n_measure"]) * p["L"] for p in probs)
    legs = {}
    for name, delay in (("window", 0), ("delayed_k16", 16)):
        ctx = hfqmc.Context(0)
        pk = [dict(p, delay=delay) for p in probs]
        ctx.stage(pk)
        ms, _, kern = timed_runs(ctx, args.steps, args.warmup)
        r = ctx.collect()
        assert all(x["status"] == 0 for x in r)
        legs[name] = dict(ms=ms, kernel_ms=float(np.mean(kern)), proposals_per_s=props / (ms * 1e-3),
                          us_per_proposal_of_a_chain=float(np.mean(kern)) * 1e3 / (2200 * 160),
                          max_drift=max(x["max_drift"] for x in r), plan=list(ctx.plan(160, delay)[:2]))
        ctx.close()
    _line("HF-QMC spin-flip proposals/s (L=160, G in device memory)", legs["window"]["proposals_per_s"], "proposals/s",
          args.steps, args.warmup, legs["window"]["ms"],
          {"workload": "128 impurities at L=160 (serving generator: U=8, dtau=0.25, open 64-site chain centre site, "
                       "mu_eff~U[-1,1]), 200+2000 sweeps, fp64", "proposals_per_step": props}, legs=legs)


def bench_lattice(args, name):
    from paper_1006_2716_amd import hfqmc, workloads
    if name == "trapped":
        probs = workloads.trapped_21x21()
        legs = [("fp64", hfqmc.FP64, 0)]
        desc = "21x21 trap V0=0.05, U=8, beta=10, L=40, AF seed h=0.1, 325 sites n>1e-3, 1000+10000 sweeps"
    else:
        probs = workloads.slab_41x41()
        legs = [("fp64", hfqmc.FP64, 0), ("mixed", hfqmc.MIXED, 0)]
        desc = "41x41 trap V0=0.02, U=8, beta=16, L=80, mu_eff for ~1000 atoms, AF seed, 1281 sites, 1000+10000 sweeps"
    props = sum((p["n_warmup"] + p["n_measure"]) * p["L"] for p in probs)
    res = {}
    ref = None
    for leg, prec, k in legs:
        ctx = hfqmc.Context(0, precision=prec)
        pk = [dict(p, delay=k) for p in probs]
        ctx.stage(pk)
        ms, _, _ = timed_runs(ctx, 1, 0)
        r = ctx.collect()
        ok = [i for i, x in enumerate(r) if x["status"] == 0]
        res[leg] = dict(proposals_per_s=props / (ms * 1e-3), ms=ms, max_drift=max(r[i]["max_drift"] for i in ok),
                        atoms=float(sum(r[i]["n_up"] + r[i]["n_dn"] for i in ok)), failed=len(r) - len(ok),
                        recoveries=int(sum(x["recoveries"] for x in r)))
        if ref is None:
            ref = r
        else:
            res[leg]["max_g_shift_vs_fp64"], res[leg]["max_g_shift_sigma"] = _g_shift([r[i] for i in ok],
                                                                                     [ref[i] for i in ok])
        ctx.close()
    _line(f"HF-QMC spin-flip proposals/s ({name} lattice)", res["fp64"]["proposals_per_s"], "proposals/s", 1, 0,
          res["fp64"]["ms"], {"workload": desc, "n_impurities": len(probs), "proposals": props}, legs=res)


def _lattice_flops(layer, n_layers):
    """Algorithmic flops of one (spin, frequency) matrix of the layered lattice
    Green function: a Gauss-Jordan inverse per layer (8 b^3) forward, two
    complex b x b products per layer (16 b^3) backward."""
    b3 = float(layer) ** 3
    return 8.0 * b3 * n_layers + 16.0 * b3 * (n_layers - 1)


def bench_rdmft(args):
    """One RDMFT iteration of the 21 x 21 trap (lattice Green function at 500
    frequencies, Weiss functions, the 325-site solve, self-energy), the same
    with 2 chains per site, and one iteration of the 41 x 41 trap (1281 sites
    at L = 80)."""
    import torch
    from paper_1006_2716_amd import hfqmc, workloads
    from paper_1006_2716_amd.rdmft import RDMFT
    nf = 500
    parts = {}
    for name, n, V0, U, beta, L, mu_eff in (("21x21", 21, 0.05, 8.0, 10.0, 40, 0.0),
                                            ("41x41", 41, 0.02, 8.0, 16.0, 80, workloads.C5_MU_EFF)):
        hop, eps, sites = workloads.trapped_lattice(n, V0, beta, mu_eff, 0.1)
        ctx = hfqmc.Context(0)
        r = RDMFT(ctx, hop, n, eps, mu_eff, U, beta, L, n_freq=nf)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        r.weiss(sites)  # warm-up
        torch.cuda.synchronize()
        reps = max(1, args.steps)
        green_ms, weiss_ms = 0.0, 0.0
        for _ in range(reps):  # events on the context's stream (torch's current one)
            ev[0].record()
            r.lat.green(nf, beta, mu_eff, r.eps, r.sigma, out=r.gloc)
            ev[1].record()
            r.lat.weiss(nf, beta, mu_eff, L, r.eps, r.gloc, r.sigma, sites)
            ev[2].record()
            torch.cuda.synchronize()
            green_ms += ev[0].elapsed_time(ev[1]) / reps
            weiss_ms += ev[1].elapsed_time(ev[2]) / reps
        flops = 2 * nf * _lattice_flops(n, n)
        leg = dict(sites=n * n, solved_sites=int(len(sites)), n_freq=nf, lattice_green_ms=green_ms,
                   weiss_ms=weiss_ms, lattice_tflops=flops / (green_ms * 1e-3) / 1e12,
                   lattice_flops=flops)
        # one full iteration of each trap (the 41 x 41 one solves 1281 sites at L = 80), after an untimed
        # short one on a throwaway loop (the first solve of a process loads the sweep kernels)
        rw = RDMFT(ctx, hop, n, eps, mu_eff, U, beta, L, n_freq=nf, lattice=r.lat)
        rw.iterate(sites, n_warmup=2, n_measure=4, seed=1, n_bins=2)
        rw.close()
        it = r.iterate(sites, n_warmup=1000, n_measure=10000, seed=2 if name == "21x21" else 5, timing=True)
        props = int(sum(x["proposals"] for x in it["results"]))
        leg.update(iteration_ms=sum(it["ms"].values()), steps_ms=it["ms"], proposals=props,
                   atoms=float(it["density"].sum()))
        if name == "21x21":
            # the same iteration with every site split into 2 chains (each with the full warm-up and half
            # the measured sweeps): 650 units fill the GPU better than 325
            r2 = RDMFT(ctx, hop, n, eps, mu_eff, U, beta, L, n_freq=nf, lattice=r.lat)
            it2 = r2.iterate(sites, n_warmup=1000, n_measure=10000, seed=2, timing=True, n_chains=2)
            r2.close()
            leg["two_chains"] = dict(iteration_ms=sum(it2["ms"].values()), steps_ms=it2["ms"],
                                     proposals=int(sum(x["proposals"] for x in it2["results"])),
                                     atoms=float(it2["density"].sum()))
        parts[name] = leg
        r.close()
        ctx.close()
    c2 = parts["21x21"]
    it_ms = c2["iteration_ms"]
    _line("RDMFT iteration, 21x21 trap: proposals/s of the whole iteration", c2["proposals"] / (it_ms * 1e-3),
          "proposals/s", 1, 0, it_ms,
          {"workload": "21x21 open trap V0=0.05, U=8, beta=10, L=40, AF seed h=0.1 in the site energies, "
                       "lattice Green function at 500 Matsubara frequencies x 2 spins, Weiss functions of the "
                       "325 sites with n>1e-3, their 1000+10000-sweep solve, self-energy update"},
          lattice_roofline={"bound": "alu", "kernel": "hfqmc::rgf_kernel<32>",
                            "achieved": round(c2["lattice_tflops"], 3), "peak": 78.6, "unit": "TFLOP/s",
                            "frac": round(c2["lattice_tflops"] / 78.6, 4), "traffic": lattice_traffic(),
                            "hbm_gbps": (round(lattice_traffic() / (c2["lattice_green_ms"] * 1e-3) / 1e9, 1)
                                         if lattice_traffic() else None)},
          parts=parts)


def bench_trotter(args):
    """dtau -> 0 for the 21 x 21 trap's 325 sites: L = 32, 40, 50 (dtau =
    0.3125, 0.25, 0.2) in one uneven-L batch, 200 + 2000 sweeps, then the fit
    even in dtau per site."""
    from paper_1006_2716_amd import hfqmc, workloads
    from paper_1006_2716_amd.trotter import solve_extrapolated
    Ls = (32, 40, 50)
    by_L = {L: workloads.trapped_square(21, 0.05, 8.0, 10.0, L, 0.0, 0.1, 200, 2000, seed=2)[0] for L in Ls}
    props = sum((p["n_warmup"] + p["n_measure"]) * p["L"] for L in Ls for p in by_L[L])
    ctx = hfqmc.Context(0)
    solve_extrapolated(ctx, {L: v[:4] for L, v in by_L.items()})  # warm-up (kernel load)
    t0 = time.perf_counter()
    est, per_L = solve_extrapolated(ctx, by_L, order=1)
    ms = (time.perf_counter() - t0) * 1e3
    ctx.close()
    atoms = {L: float(sum(r["n_up"] + r["n_dn"] for r in per_L[L])) for L in Ls}
    atoms0 = float(sum(e["n_up"] + e["n_dn"] for e in est))
    dmax = max(abs(e["docc"] - r["docc"]) for e, r in zip(est, per_L[40]))
    _line("dtau->0 extrapolation, 21x21 trap (3 grids, one batch): proposals/s", props / (ms * 1e-3),
          "proposals/s", 1, 0, ms,
          {"workload": "21x21 trap V0=0.05, U=8, beta=10, AF seed, 325 sites, L in {32,40,50} in one uneven-L "
                       "batch, 200+2000 sweeps, weighted fit c0 + c1 dtau^2 per site and observable",
           "proposals": props},
          atoms_by_L=atoms, atoms_extrapolated=atoms0, max_docc_shift_vs_L40=dmax)


def bench_thermo(args):
    """Entropy from dS/dmu = dN/dT on a 13 x 13 trap (V0 = 0.25, U = 10,
    dtau = 0.1, T = 1/(4.2) .. 1/(3.8)): converged RDMFT at 45 chemical
    potentials and two temperatures, from the empty system up to half filling
    at the centre, seeded with a staggered field; central and average entropy
    per particle (with their statistical errors) and the staggered
    magnetization."""
    from paper_1006_2716_amd import hfqmc, workloads
    from paper_1006_2716_amd.thermo import entropy_scan, staggered_magnetization
    n, V0, U, dtau = 13, 0.25, 10.0, 0.1
    Hu, Hd, coords = workloads.trapped_square_onebody(n, n, V0, 0.0, 0.1)
    hop = Hu - np.diag(np.diag(Hu))
    eps_seed = np.stack([np.diag(Hu), np.diag(Hd)])
    eps = np.stack([0.5 * (eps_seed[0] + eps_seed[1])] * 2)  # the trap alone: the seed field cancels
    mus = np.linspace(-11.0, 0.0, 45)
    sites = np.arange(n * n, dtype=np.int32)
    ctx = hfqmc.Context(0)
    t0 = time.perf_counter()
    r = entropy_scan(ctx, hop, n, eps, eps_seed, U, mus, 38, 42, dtau, sites, 100, args.thermo_sweeps, seed=5,
                     n_freq=500, tol=5e-3, max_iter=args.thermo_iters, n_bins=16, mu_group=args.mu_group)
    ms = (time.perf_counter() - t0) * 1e3
    ctx.close()
    c = n * n // 2
    N = float(r["n_hi"][-1].sum() + r["n_lo"][-1].sum()) / 2.0
    dens = 0.5 * (r["n_lo"][-1] + r["n_hi"][-1])
    m = staggered_magnetization(dens, coords)
    _line("entropy scan, 13x13 trap (45 mu x 2 T, converged RDMFT): proposals/s", r["proposals"] / (ms * 1e-3),
          "proposals/s", 1, 0, ms,
          {"workload": "13x13 open trap V0=0.25, U=10, dtau=0.1, L=38/42, mu-U/2 from -11 to 0 (45 points), "
                       "staggered seed 0.1 in the first iteration at each point, "
                       f"100+{args.thermo_sweeps} sweeps, <={args.thermo_iters} iterations per point, "
                       f"{args.mu_group} chemical potential(s) per solver batch",
           "proposals": r["proposals"], "rdmft_iterations": int(sum(r["iterations"]))},
          T=r["T"], atoms=N, entropy_central=float(r["s"][-1][c]), entropy_central_err=float(r["s_err"][-1][c]),
          entropy_per_particle=float(r["s"][-1].sum() / N),
          entropy_per_particle_err=float(np.sqrt((r["s_err"][-1] ** 2).sum()) / N),
          m_stag_central=float(m[c]), m_stag_max=float(np.abs(m).max()),
          # largest change of a spin density (the loops' 5e-3 tolerance) and of n_up + n_dn in each (mu, T)
          # point's last iteration
          points=int(r["last_change"].shape[0]), points_below_tol=int(np.sum(r["last_change"][:, 0] < 5e-3)),
          last_change_median=float(np.nanmedian(r["last_change"][:, 0])),
          last_change_max=float(np.nanmax(r["last_change"][:, 0])),
          last_change_total_median=float(np.nanmedian(r["last_change"][:, 1])),
          last_change_total_max=float(np.nanmax(r["last_change"][:, 1])))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="headline", choices=["headline", "uneven", "long", "serving", "serving_chains",
                                                                "trapped", "slab", "rdmft", "trotter", "thermo", "all"])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-single", action="store_true", help="skip the single-impurity comparison")
    ap.add_argument("--delay", type=int, default=0,
                    help="update kind: 0 the library's choice for L (default), 1 rank-one, 2..32 delayed rank-k")
    ap.add_argument("--no-serving", action="store_true", help="headline: skip the serving-latency leg")
    ap.add_argument("--no-workloads", action="store_true",
                    help="headline: skip the uneven-L, L = 160 and slab legs (each run in a process of its own)")
    ap.add_argument("--tune-cache", default=None, help="serving: a tuning cache fixing kernel shapes per padded L")
    ap.add_argument("--shape", default=None, metavar="RT,K",
                    help="headline: force the L = 64 kernel shape (tile-rows per wave, k: 0 window, 1 rank-one, "
                         ">1 delayed) through a temporary tuning cache")
    ap.add_argument("--mixed", action="store_true", help="fp32 products in the window flush or the delayed updates")
    ap.add_argument("--graph", action="store_true", help="replay the pass from a captured hipGraph")
    ap.add_argument("--step-ms", type=float, default=8.0, help="serving: target step duration")
    ap.add_argument("--quantum", type=int, default=0, help="serving: fixed proposals per request per step")
    ap.add_argument("--serve-chains", type=int, default=1, help="serving: chains per L = 160 request")
    ap.add_argument("--thermo-sweeps", type=int, default=2000, help="thermo: measured sweeps per solve")
    ap.add_argument("--thermo-iters", type=int, default=5, help="thermo: most RDMFT iterations per (mu, T) point")
    ap.add_argument("--mu-group", type=int, default=9,
                    help="thermo: chemical potentials whose loops share one solver batch")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this engine runs on one GPU; multi-GPU sharding is a design "
                                   "note only (impurities shard with no exchange), not built"}))
        sys.exit(2)
    if args.workload == "all":
        # every leg in a process of its own: kernel-class concurrency depends
        # on how the process's streams map onto its few hardware queues, which
        # shifts with the streams earlier contexts created (measured: serving
        # p50 122 ms first in a process, 235 ms after the uneven leg); this
        # process never touches the GPU itself
        import subprocess
        rc = 0
        for n in ["uneven", "long", "serving", "serving_chains", "trapped", "slab", "rdmft", "trotter", "thermo"]:
            print(f"== {n}", file=sys.stderr, flush=True)
            cmd = [sys.executable, os.path.abspath(__file__), "--workload", n, "--steps", str(args.steps), "--warmup",
                   str(args.warmup), "--step-ms", str(args.step_ms), "--quantum", str(args.quantum)]
            rc = subprocess.run(cmd).returncode or rc
        sys.exit(rc)
    if args.workload != "headline":
        names = [args.workload]
        for n in names:
            print(f"== {n}", file=sys.stderr, flush=True)
            if n == "uneven":
                bench_uneven(args)
            elif n == "long":
                bench_long(args)
            elif n == "serving":
                bench_serving(args)
            elif n == "serving_chains":
                bench_serving(argparse.Namespace(**dict(vars(args), serve_chains=4)))
            elif n == "rdmft":
                bench_rdmft(args)
            elif n == "trotter":
                bench_trotter(args)
            elif n == "thermo":
                bench_thermo(args)
            else:
                bench_lattice(args, n)
        return

    import torch
    from paper_1006_2716_amd import hfqmc, workloads

    probs = workloads.chain_batch_L64()
    for p in probs:
        p["delay"] = args.delay
    n_imp = len(probs)
    L = probs[0]["L"]
    tune = None
    if args.shape:
        import tempfile
        rt_f, k_f = (int(x) for x in args.shape.split(","))
        fd, tune = tempfile.mkstemp(suffix=".json")
        with os.fdopen(fd, "w") as f:
            json.dump({"arch": "gfx950", "entries": [{"precision": "mixed" if args.mixed else "fp64", "L_padded": 64,
                                                       "rt": rt_f, "k": k_f, "proposals_per_s": 1.0}]}, f)
    ctx = hfqmc.Context(0, precision=hfqmc.MIXED if args.mixed else hfqmc.FP64, tune_cache=tune)
    if tune:
        os.unlink(tune)  # read at context creation
    ws = ctx.alloc_workspace(probs)
    ctx.stage(probs, ws)
    rt, k, _ = ctx.plan(L, args.delay)
    # kernel time from the sweep kernel's own events (the whole pass when
    # replayed from a graph)
    ms_per_step, step_ms, kern_ms = timed_runs(ctx, args.steps, args.warmup, graph=args.graph)

    res = ctx.collect()
    proposals = sum(r["proposals"] for r in res)
    accepts = sum(r["accepts"] for r in res)
    assert all(r["status"] == 0 for r in res), "non-finite result"
    p_acc = accepts / proposals
    value = proposals / (ms_per_step * 1e-3)

    window = k == 0
    kbar = 0.0 if k <= 1 else (k - 1) / 2.0  # mean pending updates while appending
    flops_launch = proposals * algorithmic_flops(L, p_acc, kbar=kbar)
    kavg = float(np.mean(kern_ms))
    achieved = flops_launch / (kavg * 1e-3) / 1e12
    if window:
        dk = 4 if args.mixed else 3
        kname = f"hfqmc::window_kernel<WCfg<64,{rt},{1 if args.mixed else 0}>>"
        # the window kernel's update flops run on the matrix cores: fp64 MFMA
        # (78.6 TFLOP/s on MI355X, the same figure as the fp64 vector peak),
        # fp32 MFMA when the flush forms fp32 products
        bound, peak = "mfma", (FP32_MFMA_PEAK_TFLOPS if args.mixed else FP64_VECTOR_PEAK_TFLOPS)
    else:
        dk = 0 if k <= 1 else (2 if args.mixed else 1)
        kname = f"hfqmc::sweep_kernel<Cfg<64,{rt},{dk}>>"
        bound, peak = "alu", FP64_VECTOR_PEAK_TFLOPS
    traffic = kernel_traffic(kname) if not args.graph else None
    roofline = dict(bound=bound, achieved=round(achieved, 3), peak=peak, unit="TFLOP/s",
                    frac=round(achieved / peak, 4), traffic=traffic, kernel=kname, kernel_avg_ms=round(kavg, 4),
                    flops_per_launch=flops_launch)

    out = {
        "metric": "HF-QMC spin-flip proposals/s (batched impurities, L=64) + p99 solve latency",
        "value": value,
        "unit": "proposals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        # wall time of one whole batch solve (a step); the per-request
        # latency of the serving stream is p50/p99_request_latency_ms
        "p50_solve_ms": float(np.percentile(step_ms, 50)),
        "p99_solve_ms": float(np.percentile(step_ms, 99)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if not args.mixed else "f64+f32 (update products)",
        "data": "synthetic",
        "config": {"workload": "512 impurities x L=64 (beta=8, dtau=0.125), U~U[4,12], open 64-site chain "
                               "centre-site Weiss at mu_eff~U[-1,1], 200+2000 sweeps, "
                               + ("window updates (16 slices, MFMA flush)" if window else
                                  ("rank-one SM updates" if k <= 1 else f"delayed rank-{k} updates"))
                               + (", fp32 products" if args.mixed else ", fp64"),
                   "n_impurities": n_imp, "L": L, "sweeps": 2200, "recompute_every": RECOMPUTE_EVERY,
                   "proposals_per_step": proposals, "accept_rate": round(p_acc, 4), "delay": k,
                   "tile_rows_per_wave": rt, "graph": bool(args.graph)},
        "roofline": roofline,
        # what bounds the launch: the impurity with the most accepted flips is
        # one serial Markov chain; the kernel time over its accepts is the
        # latency of one accept on the critical path
        "critical_path": {"max_accepts": int(max(r["accepts"] for r in res)),
                          "mean_accepts": float(np.mean([r["accepts"] for r in res])),
                          "ns_per_accept": round(kavg * 1e6 / max(r["accepts"] for r in res), 1)},
        "max_drift": max(r["max_drift"] for r in res),
    }
    if not args.no_single:
        single = single_impurity_rate(ctx, probs)
        out["single_impurity_path_proposals_per_s"] = single
        out["speedup_vs_single_impurity_path"] = value / single
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(probs)
    ctx.close()
    if not args.no_serving:
        # the metric's latency half: per-request p50/p99 of the serving stream,
        # measured in a process of its own (stream-to-queue mapping depends on
        # the contexts a process created before)
        import subprocess
        cp = subprocess.run([sys.executable, os.path.abspath(__file__), "--workload", "serving"], capture_output=True,
                            text=True)
        line = [x for x in cp.stdout.splitlines() if x.startswith("{")]
        if cp.returncode == 0 and line:
            srv = json.loads(line[-1])
            s = srv.get("serving", {})
            out["serving"] = {k: s.get(k) for k in ("p50_ms", "p99_ms", "p50_ms_by_L", "requests", "proposals_per_s",
                                                    "makespan_s")
                              if k in s}
            out["serving"]["workload"] = srv["config"]["workload"]
            out["p50_request_latency_ms"] = out["serving"].get("p50_ms")
            out["p99_request_latency_ms"] = out["serving"].get("p99_ms")
        else:
            out["serving"] = {"error": f"serving leg exited {cp.returncode}"}
    if not args.no_workloads:
        # the other benchmark configurations, each in a process of its own:
        # their headline figures ride on this line
        import subprocess
        out["workloads"] = {}
        for n in ("uneven", "long", "slab"):
            cp = subprocess.run([sys.executable, os.path.abspath(__file__), "--workload", n], capture_output=True,
                                text=True)
            line = [x for x in cp.stdout.splitlines() if x.startswith("{")]
            if cp.returncode != 0 or not line:
                out["workloads"][n] = {"error": f"{n} leg exited {cp.returncode}"}
                continue
            w = json.loads(line[-1])
            e = {k: w[k] for k in ("metric", "value", "unit", "ms_per_step") if k in w}
            e["workload"] = w["config"]["workload"]
            if n == "uneven":
                e["class_launch_ms_L_items"] = w["config"].get("class_launch_ms_L_items")
                mx = w.get("mixed_fp32_products", {}).get("window", {})
                e["mixed_window"] = {k: mx.get(k) for k in ("proposals_per_s", "failed", "max_drift")}
            elif n == "long":
                e["us_per_proposal_of_a_chain"] = w.get("legs", {}).get("window", {}).get("us_per_proposal_of_a_chain")
            elif n == "slab":
                mx = w.get("legs", {}).get("mixed", {})
                e["mixed"] = {k: mx.get(k) for k in ("proposals_per_s", "failed", "max_drift")}
            out["workloads"][n] = e
    print(json.dumps(out))


if __name__ == "__main__":
    main()
