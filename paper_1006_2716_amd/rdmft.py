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
                 n_freq: int = 500, mix: float = 1.0, sigma0=None):
        torch = _torch()
        self.ctx = ctx
        self.dev = f"cuda:{ctx.device}"
        self.lat = hfqmc.Lattice(ctx, hop, layer)
        self.N = self.lat.n_sites
        self.eps = torch.as_tensor(np.asarray(eps, dtype=np.float64), device=self.dev).contiguous()
        self.mu, self.U, self.beta, self.L, self.n_freq, self.mix = float(mu), float(U), float(beta), int(L), \
            int(n_freq), float(mix)
        if sigma0 is None:
            self.sigma = torch.zeros((2, self.n_freq, self.N), dtype=torch.complex128, device=self.dev)
        else:
            self.sigma = torch.as_tensor(np.asarray(sigma0, dtype=np.complex128), device=self.dev).contiguous()
        self.gloc = None

    def close(self):
        self.lat.close()

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

    def iterate(self, sites, n_warmup, n_measure, seed, n_bins=32, recompute_every=50, n_chains=0,
                sweep_offset=0, timing=False):
        """One full iteration; returns the solver results, the densities and
        (timing=True) the wall time of each step in ms."""
        torch = _torch()
        sync = (lambda: torch.cuda.synchronize(self.dev)) if timing else (lambda: None)
        t = [time.perf_counter()]
        w_iw, w_tau = self.weiss(sites)
        sync()
        t.append(time.perf_counter())
        res = self.ctx.solve(self.problems(sites, w_tau, n_warmup, n_measure, seed, n_bins, recompute_every,
                                           n_chains, sweep_offset))
        t.append(time.perf_counter())
        dens = self.update(sites, w_iw, res)
        sync()
        t.append(time.perf_counter())
        out = dict(results=res, density=dens, weiss_tau=w_tau)
        if timing:
            out["ms"] = dict(lattice_and_weiss=1e3 * (t[1] - t[0]), solve=1e3 * (t[2] - t[1]),
                             sigma=1e3 * (t[3] - t[2]))
        return out
