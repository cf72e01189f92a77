"""Real-space DMFT iterations on one GPU, as a client of the C ABI.

One iteration (the paper's self-consistency, Eq. (2) and the impurity problem
of each site): lattice Green function from the current self-energy, Weiss
functions of the solved sites and their tau samples, one batched HF-QMC solve,
new self-energy.  Every step runs in the library's kernels; this module only
moves arrays between the calls (the solver takes and returns host arrays).
"""
from __future__ import annotations

import time

import numpy as np

from . import hfqmc


def _torch():
    import torch  # noqa: PLC0415
    return torch


class RDMFT:
    """hop (N, N) real symmetric hopping, layer sites per layer (see
    hfqmc_lattice_create), eps (2, N) site energies, mu the chemical potential
    of the Hartree-shifted levels (mu - U/2), sigma relative to them."""

    def __init__(self, ctx: hfqmc.Context, hop, layer: int, eps, mu: float, U: float, beta: float, L: int,
                 n_freq: int = 500, mix: float = 1.0, sigma0=None, lattice: hfqmc.Lattice | None = None):
        torch = _torch()
        self.ctx = ctx
        self.dev = f"cuda:{ctx.device}"
        self.own_lattice = lattice is None
        self.lat = hfqmc.Lattice(ctx, hop, layer) if lattice is None else lattice
        self.N = self.lat.n_sites
        self.eps = torch.as_tensor(np.asarray(eps, dtype=np.float64), device=self.dev).contiguous()
        self.mu, self.U, self.beta, self.L, self.n_freq, self.mix = float(mu), float(U), float(beta), int(L), \
            int(n_freq), float(mix)
        if sigma0 is None:
            self.sigma = torch.zeros((2, self.n_freq, self.N), dtype=torch.complex128, device=self.dev)
        else:
            self.sigma = torch.as_tensor(np.asarray(sigma0, dtype=np.complex128), device=self.dev).contiguous()
        self.gloc = None
        self.fields = {}  # site -> final fields of its last solve (used with keep_fields)

    def close(self):
        if self.own_lattice:
            self.lat.close()

    def set_eps(self, eps):
        """New site energies (e.g. the seed field switched off after the first iteration)."""
        self.eps = _torch().as_tensor(np.asarray(eps, dtype=np.float64), device=self.dev).contiguous()

    def weiss(self, sites):
        """Lattice Green function and Weiss functions of `sites` from the
        current self-energy: (weiss_iw (2, n_freq, n_sel) on the device,
        weiss_tau (n_sel, 2, L) on the host)."""
        self.gloc = self.lat.green(self.n_freq, self.beta, self.mu, self.eps, self.sigma, out=self.gloc)
        w_iw, w_tau = self.lat.weiss(self.n_freq, self.beta, self.mu, self.L, self.eps, self.gloc, self.sigma,
                                     sites)
        return w_iw, w_tau.cpu().numpy()

    def problems(self, sites, weiss_tau, n_warmup, n_measure, seed, n_bins=32, recompute_every=50, n_chains=0,
                 sweep_offset=0):
        return [dict(L=self.L, beta=self.beta, U=self.U, weiss=weiss_tau[j], n_warmup=n_warmup,
                     n_measure=n_measure, recompute_every=recompute_every, n_bins=n_bins, seed=seed,
                     site=int(sites[j]), sweep_offset=sweep_offset, n_chains=n_chains) for j in range(len(sites))]

    def update(self, sites, weiss_iw, results):
        """New self-energy at `sites` from the solver's results."""
        torch = _torch()
        gimp = np.stack([np.stack([r["g_up"], r["g_dn"]]) for r in results])
        dens = np.array([[r["n_up"], r["n_dn"]] for r in results], dtype=np.float64)
        g_dev = torch.as_tensor(gimp, device=self.dev).contiguous()
        d_dev = torch.as_tensor(dens, device=self.dev).contiguous()
        self.lat.sigma_update(self.n_freq, self.beta, self.mu, self.U, self.L, self.eps, sites, weiss_iw, g_dev,
                              d_dev, self.mix, self.sigma)
        return dens

    def prepare(self, sites, n_warmup, n_measure, seed, n_bins=32, recompute_every=50, n_chains=0,
                sweep_offset=0, keep_fields=False):
        """First half of an iteration: lattice Green function, Weiss functions
        and the solver problems of the live sites.  A site whose Weiss
        function is empty or full to rounding (g(0+) within 1e-12 of 0 or 1,
        far below or above the band) is not solved: its density is the Weiss
        function's and its self-energy stays.  keep_fields: a site solved
        before starts from its last final fields (all its chains) instead of
        drawn ones, so a short warm-up suffices."""
        sites = np.asarray(sites, dtype=np.int32)
        w_iw, w_tau = self.weiss(sites)
        g0 = w_tau[:, :, 0]
        live = np.all((g0 > 1e-12) & (g0 < 1.0 - 1e-12), axis=1)
        idx = np.nonzero(live)[0]
        probs = self.problems(sites[idx], w_tau[idx], n_warmup, n_measure, seed, n_bins, recompute_every, n_chains,
                              sweep_offset)
        if keep_fields:
            for p in probs:
                f = self.fields.get(p["site"])
                if f is not None:
                    p["init_fields"] = f
        return dict(sites=sites, w_iw=w_iw, w_tau=w_tau, live=live, idx=idx, problems=probs)

    def finish(self, st, res):
        """Second half: the new self-energy from the solver's results `res` (in
        the order of st['problems']); returns the iteration's output."""
        torch = _torch()
        sites, live, idx, w_tau = st["sites"], st["live"], st["idx"], st["w_tau"]
        dens = 1.0 - w_tau[:, :, 0].copy()
        dens_err = np.zeros_like(dens)
        total_err = np.zeros(len(sites))  # error of n_up + n_dn from the bins (the spins are correlated)
        if len(idx):
            w_iw = st["w_iw"]
            sub = w_iw if live.all() else w_iw[:, :, torch.as_tensor(idx, device=self.dev)].contiguous()
            dens[idx] = self.update(sites[idx], sub, res)
            dens_err[idx] = np.array([[x["n_up_err"], x["n_dn_err"]] for x in res])
            for j, x in zip(idx, res):
                self.fields[int(sites[j])] = x["fields"].copy()
            L = self.L
            for j, x in zip(idx, res):
                tot = x["bins"][:, 2 * L + 2] + x["bins"][:, 2 * L + 3]
                total_err[j] = tot.std(ddof=1) / np.sqrt(tot.size)
        return dict(results=res, density=dens, density_err=dens_err, total_err=total_err, weiss_tau=w_tau,
                    solved=live)

    def iterate(self, sites, n_warmup, n_measure, seed, n_bins=32, recompute_every=50, n_chains=0,
                sweep_offset=0, timing=False, keep_fields=False):
        """One full iteration (prepare, one batched solve, finish); returns the
        solver results (live sites), the densities of all listed sites and
        (timing=True) the wall time of each step in ms."""
        torch = _torch()
        sync = (lambda: torch.cuda.synchronize(self.dev)) if timing else (lambda: None)
        t = [time.perf_counter()]
        st = self.prepare(sites, n_warmup, n_measure, seed, n_bins, recompute_every, n_chains, sweep_offset,
                          keep_fields)
        sync()
        t.append(time.perf_counter())
        res = self.ctx.solve(st["problems"]) if st["problems"] else []
        t.append(time.perf_counter())
        out = self.finish(st, res)
        sync()
        t.append(time.perf_counter())
        if timing:
            out["ms"] = dict(lattice_and_weiss=1e3 * (t[1] - t[0]), solve=1e3 * (t[2] - t[1]),
                             sigma=1e3 * (t[3] - t[2]))
        return out

    def converge(self, sites, n_warmup, n_measure, seed, tol=2e-3, max_iter=20, eps_after=None,
                 n_warmup_next=None, **kw):
        """Iterate until the largest density change between iterations is below
        tol (or max_iter).  eps_after (e.g. without the seed field) replaces
        the site energies after the first iteration.  n_warmup_next: later
        iterations start every site from its previous final fields with this
        many warm-up sweeps.  Returns the last iteration's output with
        'history' (largest change of a spin density per iteration),
        'history_total' (the same for n_up + n_dn) and 'proposals_all'
        (solver proposals of every iteration)."""
        prev, hist, hist_tot, total = None, [], [], 0
        for it in range(max_iter):
            if it > 0 and n_warmup_next is not None:
                out = self.iterate(sites, n_warmup_next, n_measure, seed + it, keep_fields=True, **kw)
            else:
                out = self.iterate(sites, n_warmup, n_measure, seed + it, **kw)
            total += _proposals(out["results"])
            if it == 0 and eps_after is not None:
                self.set_eps(eps_after)
            d = out["density"]
            if prev is not None:
                hist.append(float(np.max(np.abs(d - prev))))
                hist_tot.append(float(np.max(np.abs(d.sum(axis=1) - prev.sum(axis=1)))))
                if hist[-1] < tol:
                    break
            prev = d
        out["history"] = hist
        out["history_total"] = hist_tot
        out["proposals_all"] = total
        return out


def _proposals(results):
    return int(sum(int(x["proposals"]) for x in results))


def converge_together(loops, sites, n_warmup, n_measure, seeds, tol=2e-3, max_iter=20, eps_after=None,
                      n_warmup_next=None, **kw):
    """converge() for several independent loops (e.g. two temperatures) that
    share one batched solve per iteration: the solver sees all their live
    sites at once, which fills the GPU better than one loop alone.  Each loop
    stops once its own density change is below tol (or at max_iter).
    seeds: one per loop; n_warmup_next as in converge().  Returns the outputs
    of every loop's last iteration, with 'history', 'history_total' and
    'proposals_all' as in converge()."""
    ctx = loops[0].ctx
    prev = [None] * len(loops)
    hist = [[] for _ in loops]
    hist_tot = [[] for _ in loops]
    total = [0] * len(loops)
    outs = [None] * len(loops)
    active = list(range(len(loops)))
    for it in range(max_iter):
        warm = it > 0 and n_warmup_next is not None
        states = [loops[k].prepare(sites, n_warmup_next if warm else n_warmup, n_measure, seeds[k] + it,
                                   keep_fields=warm, **kw) for k in active]
        batch = [p for st in states for p in st["problems"]]
        res = ctx.solve(batch) if batch else []
        pos = 0
        still = []
        for k, st in zip(active, states):
            m = len(st["problems"])
            outs[k] = loops[k].finish(st, res[pos:pos + m])
            total[k] += _proposals(res[pos:pos + m])
            pos += m
            if it == 0 and eps_after is not None:
                loops[k].set_eps(eps_after)
            d = outs[k]["density"]
            done = False
            if prev[k] is not None:
                hist[k].append(float(np.max(np.abs(d - prev[k]))))
                hist_tot[k].append(float(np.max(np.abs(d.sum(axis=1) - prev[k].sum(axis=1)))))
                done = hist[k][-1] < tol
            prev[k] = d
            if not done:
                still.append(k)
        active = still
        if not active:
            break
    for k in range(len(loops)):
        outs[k]["history"] = hist[k]
        outs[k]["history_total"] = hist_tot[k]
        outs[k]["proposals_all"] = total[k]
    return outs
