"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

* forced-flip sequences and from-scratch Dyson solves: G to 1e-10 (fp64);
* full Markov chains: both sides draw the same Philox stream, so the field
  trajectories coincide (up to a rounding tie |u - R| ~ 1e-16, never seen)
  and the observables agree to rounding; compared element by element;
* statistics against exact enumeration and the isolated atom;
* the full-size L = 64 batch at the benchmark's launch configuration,
  sampled impurities recomputed by the oracle.
"""
import numpy as np
import pytest

import oracle
from oracle import exact as ex
from paper_1006_2716_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL_G = 1e-10


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1006_2716_amd import hfqmc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hfqmc.Context(0)
    c.attach_pool(64 << 20)
    yield c
    c.close()


def _chain_problem(L, U, mu, beta, seed=21, site=0, n_warmup=10, n_measure=40, n_bins=4, h=0.0):
    A = wl.chain_adjacency(24)
    out = []
    for sigma in (+1, -1):
        H = -A - (mu + sigma * h) * np.eye(24)
        out.append(wl.weiss_from_onebody(H, [12], beta, L)[0])
    return dict(L=L, beta=beta, U=U, weiss=np.stack(out), n_warmup=n_warmup, n_measure=n_measure,
                recompute_every=50, n_bins=n_bins, seed=seed, site=site)


# --------------------------------------------------------------- forced flips
@pytest.mark.parametrize("L", [1, 5, 16, 20, 40, 64, 80, 96, 128, 131, 160])
def test_forced_flips_match_oracle(ctx, L):
    print(f"forced flips L={L}", flush=True)
    p = _chain_problem(L, U=6.0, mu=0.3, beta=0.25 * L, h=0.2)
    lam = oracle.lam(p["beta"] / L, p["U"])
    rng = np.random.default_rng(L)
    s = rng.choice([-1, 1], L).astype(np.int8)
    slices = np.concatenate([rng.integers(0, L, size=2 * L + 3), [L - 1, L - 1, 0]]).astype(np.int32)
    site = ctx.site(L, n_bins=p["n_bins"])
    try:
        site.define(p)
        site.set_fields(s)
        G0u = oracle.dyson(p["weiss"][0], lam, 1, s)
        G0d = oracle.dyson(p["weiss"][1], lam, -1, s)
        assert np.max(np.abs(site.green(0) - G0u)) < TOL_G
        assert np.max(np.abs(site.green(1) - G0d)) < TOL_G
        ratios = site.force_flips(slices)
        Gu, Gd, s_fin, r_ref = oracle.force_flips(p["weiss"][0], p["weiss"][1], lam, s, slices)
        assert np.max(np.abs(site.green(0) - Gu)) < TOL_G
        assert np.max(np.abs(site.green(1) - Gd)) < TOL_G
        assert np.allclose(ratios, r_ref, rtol=1e-10, atol=0)
        assert np.array_equal(site.fields(), s_fin)
        drift = site.recompute()
        assert drift < 1e-9
        assert np.max(np.abs(site.green(0) - oracle.dyson(p["weiss"][0], lam, 1, s_fin))) < TOL_G
    finally:
        site.close()


# --------------------------------------------------------------- trajectories
def _compare_runs(gpu, ref, probs, tol=1e-9):
    for p, g, r in zip(probs, gpu, ref):
        L = p["L"]
        assert g["status"] == 0
        assert np.array_equal(g["fields"], r["fields"]), f"L={L}: field trajectories differ"
        assert g["proposals"] == r["proposals"] and g["accepts"] == r["accepts"]
        assert np.max(np.abs(g["bins"] - r["bins"])) < tol, f"L={L}"
        s = oracle.summarize(r["bins"], L)
        assert abs(g["n_up"] - s["n_up"]) < tol and abs(g["docc"] - s["docc"]) < tol
        assert g["max_drift"] < 1e-8


def test_plain_4x4_trajectories(ctx):
    print("plain 4x4", flush=True)
    probs = wl.plain_4x4(n_warmup=20, n_measure=200)
    gpu = ctx.solve(probs)
    ref = oracle.run(probs, n_threads=8)
    _compare_runs(gpu, ref, probs)


def test_uneven_L_batch_trajectories(ctx):
    print("uneven batch", flush=True)
    Ls = [1, 3, 16, 17, 20, 32, 40, 48, 63, 64, 65, 80, 96, 100, 112, 128, 129, 150, 160]
    probs = [_chain_problem(L, U=4.0 + 0.5 * i, mu=0.1 * i - 0.5, beta=min(0.2 * L, 10.0), seed=5, site=i,
                            n_warmup=5, n_measure=60, n_bins=6) for i, L in enumerate(Ls)]
    for p in probs[::3]:
        p["recompute_every"] = 7  # several recomputes inside the run
    gpu = ctx.solve(probs)
    ref = oracle.run(probs, n_threads=8)
    _compare_runs(gpu, ref, probs)


def test_given_initial_fields_and_sweep_offset(ctx):
    p = _chain_problem(40, U=8.0, mu=0.0, beta=10.0, n_warmup=3, n_measure=24, n_bins=3)
    p["init_fields"] = np.where(np.arange(40) % 3 == 0, -1, 1).astype(np.int8)
    p["sweep_offset"] = 12345
    gpu = ctx.solve([p])
    ref = oracle.run([p])
    _compare_runs(gpu, ref, [p])


@pytest.mark.parametrize("L", [64, 96, 160])
def test_resume_from_saved_fields_is_bit_exact(ctx, L):
    # a chain saved after 10 sweeps (its fields) and resumed with
    # sweep_offset = 10 continues bit for bit, since both runs rebuild G from
    # scratch there (recompute_every = 10 puts a scheduled solve at that sweep)
    print(f"resume L={L}", flush=True)
    base = _chain_problem(L, U=6.0, mu=0.2, beta=0.25 * L, seed=5, site=L, n_measure=20, n_bins=4)
    base["recompute_every"] = 10
    whole = ctx.solve([dict(base, n_warmup=17)])[0]
    first = ctx.solve([dict(base, n_warmup=4, n_measure=6, n_bins=2)])[0]
    resumed = dict(base, n_warmup=7, init_fields=first["fields"].copy(), sweep_offset=10)
    rest = ctx.solve([resumed])[0]
    assert np.array_equal(whole["fields"], rest["fields"])
    assert np.array_equal(whole["bins"], rest["bins"])  # bitwise
    for k in ("n_up", "n_dn", "docc"):
        assert whole[k] == rest[k], k
    for k in ("accepts", "proposals"):  # warm-up included: the two legs add up
        assert whole[k] == first[k] + rest[k], k
    _compare_runs([rest], oracle.run([resumed]), [resumed])


def test_batch_composition_does_not_change_results(ctx):
    print("composition", flush=True)
    probs = [_chain_problem(L, U=6.0, mu=0.2, beta=5.0, seed=9, site=i, n_warmup=5, n_measure=40)
             for i, L in enumerate([20, 64, 96, 40])]
    alone = ctx.solve([probs[1]])[0]
    mixed = ctx.solve(probs)[1]
    assert np.array_equal(alone["bins"], mixed["bins"])  # bitwise
    assert np.array_equal(alone["fields"], mixed["fields"])


def test_repeated_run_is_deterministic(ctx):
    probs = wl.chain_batch(n_imp=8, Ls=(32, 64), n_warmup=5, n_measure=30)
    for p in probs:
        p["n_bins"] = 5
    ctx.stage(probs)
    ctx.run()
    a = ctx.collect()
    ctx.run()
    b = ctx.collect()
    for x, y in zip(a, b):
        assert np.array_equal(x["bins"], y["bins"])


# --------------------------------------------------------------- statistics
def _z(a, b, e):
    return (a - b) / e


def test_statistics_match_enumeration(ctx):
    print("enumeration", flush=True)
    L, beta, U, mu, V, eb = 8, 2.0, 4.0, 1.0, 0.8, 0.4
    p = wl.two_site_problem(L, beta, U, mu, V, eb, h=0.2, n_warmup=500, n_measure=64000, seed=31, n_bins=32)
    lam = oracle.lam(beta / L, U)
    exact_vals, _, _ = ex.enumerate_fields(p["weiss"][0], p["weiss"][1], lam)
    g = ctx.solve([p])[0]
    zs = [_z(g["n_up"], exact_vals[2 * L + 2], g["n_up_err"]), _z(g["n_dn"], exact_vals[2 * L + 3], g["n_dn_err"]),
          _z(g["docc"], exact_vals[2 * L + 4], g["docc_err"])]
    assert max(abs(z) for z in zs) < 4.0, zs


@pytest.mark.parametrize("L", [10, 40])
def test_atom_limit(ctx, L):
    beta, U, mu, h = 3.0, 5.0, 1.8, 0.15
    p = wl.atom_problem(L, beta, U, mu, h, n_warmup=200, n_measure=12800, seed=40 + L, n_bins=32)
    g = ctx.solve([p])[0]
    ref = ex.atom_exact(beta, U, mu, h)
    for key in ("n_up", "n_dn", "docc"):
        assert abs(_z(g[key], ref[key], g[key + "_err"])) < 4.0, key


def test_U0_limit_gives_weiss(ctx):
    p = _chain_problem(32, U=0.0, mu=0.4, beta=8.0, n_warmup=2, n_measure=8, n_bins=2)
    g = ctx.solve([p])[0]
    # lambda = 0: every configuration has G = G0, so g(tau_k) is the input
    assert np.max(np.abs(g["g_up"][:32] - p["weiss"][0])) < 1e-12
    assert g["g_up"][32] == pytest.approx(1.0 - p["weiss"][0][0], abs=1e-12)


# --------------------------------------------------------------- full size
def test_full_size_L64_batch_sampled(ctx):
    """512 impurities at L = 64, 200 + 2000 sweeps, the benchmark's launch;
    three sampled impurities are recomputed by the oracle."""
    print("full-size L=64 batch", flush=True)
    probs = wl.chain_batch_L64()
    gpu = ctx.solve(probs)
    idx = [0, 255, 511]
    ref = oracle.run([probs[i] for i in idx], n_threads=3)
    _compare_runs([gpu[i] for i in idx], ref, [probs[i] for i in idx])
    acc = np.array([g["accept_rate"] for g in gpu])
    assert np.all(acc > 0.05) and np.all(acc < 0.95)
    assert all(g["status"] == 0 for g in gpu)


def test_full_size_uneven_batch_sampled(ctx):
    """512 impurities with L drawn from {32, 48, 64, 96, 128}, 200 + 2000
    sweeps, in the uneven-L benchmark's launch configuration (every class
    on its default kernel, classes concurrent); the heaviest impurity of
    each class is recomputed by the oracle."""
    print("full-size uneven batch", flush=True)
    probs = wl.chain_batch(n_imp=512, Ls=(32, 48, 64, 96, 128), seed=3)
    gpu = ctx.solve(probs)
    assert all(g["status"] == 0 for g in gpu)
    idx = [max((i for i, p in enumerate(probs) if p["L"] == L), key=lambda i: gpu[i]["accepts"])
           for L in (32, 48, 64, 96, 128)]
    ref = oracle.run([probs[i] for i in idx], n_threads=5)
    _compare_runs([gpu[i] for i in idx], ref, [probs[i] for i in idx])


def test_full_size_slab_sampled(ctx):
    """The 41 x 41 slab's 1281 sites at L = 80, 1000 + 10000 sweeps (window
    kernel, the slab benchmark's launch); the site with the most accepted
    flips and the central one are recomputed by the oracle."""
    print("full-size slab", flush=True)
    probs = wl.slab_41x41()
    gpu = ctx.solve(probs)
    assert all(g["status"] == 0 for g in gpu)
    idx = sorted({int(np.argmax([g["accepts"] for g in gpu])), len(probs) // 2})
    ref = oracle.run([probs[i] for i in idx], n_threads=2)
    _compare_runs([gpu[i] for i in idx], ref, [probs[i] for i in idx])


def test_full_size_L160_sampled(ctx):
    """128 requests of the serving generator at L = 160 as one batch, 200 +
    2000 sweeps (device-memory window kernel, the long-grid benchmark's
    launch); the impurity with the most accepted flips is recomputed by the
    oracle."""
    print("full-size L=160 batch", flush=True)
    sites, _, weiss = wl.serving_requests(n_sites=512, Ls=(160,), weights=(1,), seed=4)
    probs = [dict(L=160, beta=s["beta"], U=s["U"], weiss=weiss(s, 0), n_warmup=200, n_measure=2000,
                  recompute_every=50, n_bins=32, seed=s["seed"], site=s["site"]) for s in sites[:128]]
    gpu = ctx.solve(probs)
    assert all(g["status"] == 0 for g in gpu)
    i = int(np.argmax([g["accepts"] for g in gpu]))
    _compare_runs([gpu[i]], oracle.run([probs[i]]), [probs[i]])


def test_empty_batch(ctx):
    from paper_1006_2716_amd import hfqmc
    print("empty batch", flush=True)
    assert ctx.solve([]) == []
    assert ctx.solve_static([]) == []
    L = hfqmc.lib()
    assert L.hfqmc_solve(ctx.h, None, -1, None, 0, None) == hfqmc.EINVAL
    assert L.hfqmc_stage(ctx.h, None, 0, None, 0) == hfqmc.EINVAL  # nothing to stage
    # the context is untouched: a batch after the empty ones runs as usual
    p = _chain_problem(20, U=4.0, mu=0.1, beta=5.0, n_warmup=3, n_measure=12)
    _compare_runs(ctx.solve([p]), oracle.run([p]), [p])


def test_invalid_problems_raise(ctx):
    from paper_1006_2716_amd import hfqmc
    p = _chain_problem(16, U=4.0, mu=0.0, beta=4.0)
    bad = dict(p, L=161, weiss=np.full((2, 161), 0.5))
    with pytest.raises(hfqmc.HFQMCError):
        ctx.solve([bad])
    big = _chain_problem(150, U=4.0, mu=0.0, beta=10.0)
    with pytest.raises(hfqmc.HFQMCError):  # device-memory kernel: delay at most 16
        ctx.solve([dict(big, delay=17)])
    bad = dict(p, n_bins=1)
    with pytest.raises(hfqmc.HFQMCError):
        ctx.solve([bad])
    w = p["weiss"].copy()
    w[0, 3] = np.nan
    with pytest.raises(hfqmc.HFQMCError):
        ctx.solve([dict(p, weiss=w)])
