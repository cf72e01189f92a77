"""Thermodynamics from converged real-space DMFT solutions: density scans over
the chemical potential at two temperatures, the entropy from
dS/dmu = dN/dT (hfqmc_entropy), and staggered-magnetization profiles.

Temperatures are set through beta = L * dtau at a fixed dtau, so both
temperatures of a derivative carry the same discretisation error.
"""
from __future__ import annotations

import numpy as np

from . import hfqmc
from .rdmft import RDMFT, converge_together

# A converged loop draws solver seed base + it in its iteration it (< max_iter),
# so loop bases are spaced SEED_STRIDE apart: every (point, temperature,
# iteration) of a scan, and every bisection step of find_mu, gets a Philox key
# of its own (keys that coincide would replay the same fields and uniforms).
SEED_STRIDE = 100
MAX_TEMPERATURES = 10


def loop_seed(seed, k, a):
    """Solver seed base of chemical-potential index k at temperature index a."""
    return seed + 10 * SEED_STRIDE * k + SEED_STRIDE * a


def _check_seed_room(max_iter, n_temperatures=1):
    if max_iter > SEED_STRIDE:
        raise ValueError(f"max_iter {max_iter} > {SEED_STRIDE}: loop seeds would overlap")
    if n_temperatures > MAX_TEMPERATURES:
        raise ValueError(f"more than {MAX_TEMPERATURES} temperatures: loop seeds would overlap")


def staggered_magnetization(density, coords):
    """(-1)^(x + y) (n_up - n_dn) per site: density (sites, 2), coords (sites, 2)."""
    c = np.asarray(coords)
    d = np.asarray(density)
    return np.where(c.sum(axis=1) % 2 == 0, 1.0, -1.0) * (d[:, 0] - d[:, 1])


def density_scan(ctx, lattice, hop, layer, eps, eps_seed, U, mus, Ls, dtau, sites, n_warmup, n_measure, seed,
                 n_freq=500, tol=2e-3, max_iter=10, n_bins=16, warm_start=True, mu_group=1):
    """Converged densities at beta = L dtau for every L in Ls (several
    temperatures at a fixed dtau) and every chemical potential
    (Hartree-shifted, ascending).  The loops of mu_group consecutive chemical
    potentials and of all temperatures share one solver batch per iteration.
    The scan starts from the empty system, whose self-energy is zero, i.e.
    -U/2 relative to the Hartree-shifted levels; every loop of a group starts
    from the self-energy converged at the last chemical potential of the
    group before (warm_start) or from the empty system.  eps_seed (with a seed
    field) is used for the first iteration at every mu, eps afterwards.  The
    solver seed of (mu index k, temperature a) is loop_seed(seed, k, a), plus
    the iteration index, whatever the grouping.  Returns per L: densities (len(mus), len(sites), 2), errors
    of n_up + n_dn (len(mus), len(sites)), iteration counts, the largest
    change of a spin density and of n_up + n_dn in each point's last
    iteration (len(mus), 2) (NaN after a single iteration); and the solver
    proposals of all iterations."""
    if mu_group < 1:
        raise ValueError("mu_group must be positive")
    _check_seed_room(max_iter, len(Ls))
    N = lattice.n_sites
    empty = np.full((2, n_freq, N), -0.5 * U, dtype=np.complex128)
    sig = [empty] * len(Ls)
    dens = [np.zeros((len(mus), len(sites), 2)) for _ in Ls]
    errs = [np.zeros((len(mus), len(sites))) for _ in Ls]
    iters = [[] for _ in Ls]
    last = [np.full((len(mus), 2), np.nan) for _ in Ls]
    props = 0
    for k0 in range(0, len(mus), mu_group):
        ks = range(k0, min(k0 + mu_group, len(mus)))
        keys = [(k, a) for k in ks for a in range(len(Ls))]
        loops = [RDMFT(ctx, hop, layer, eps_seed, mus[k], U, Ls[a] * dtau, Ls[a], n_freq=n_freq,
                       sigma0=sig[a] if warm_start else empty, lattice=lattice) for k, a in keys]
        outs = converge_together(loops, sites, n_warmup, n_measure, [loop_seed(seed, k, a) for k, a in keys],
                                 tol=tol, max_iter=max_iter, eps_after=eps, n_bins=n_bins)
        for (k, a), r, o in zip(keys, loops, outs):
            dens[a][k] = o["density"]
            errs[a][k] = o["total_err"]
            iters[a].append(len(o["history"]) + 1)
            if o["history"]:
                last[a][k] = o["history"][-1], o["history_total"][-1]
            if k == ks[-1]:
                sig[a] = r.sigma.cpu().numpy()
            r.close()
        props += sum(o["proposals_all"] for o in outs)
    return dens, errs, iters, props, last


def entropy_error(mus, err_lo, err_hi, T_lo, T_hi):
    """Statistical error of each site's entropy from the densities' errors
    (independent runs at the two temperatures and at every mu), propagated
    through the central difference and the trapezoid weights: (K, sites)."""
    mus = np.asarray(mus, dtype=np.float64)
    var = (np.asarray(err_lo) ** 2 + np.asarray(err_hi) ** 2) / (T_hi - T_lo) ** 2
    h = np.diff(mus)
    out = np.zeros_like(var)
    acc = np.zeros(var.shape[1])
    for k in range(1, len(mus)):
        # s_k = sum_j w_j g_j with w_0 = h_0/2, w_j = (h_j-1 + h_j)/2, w_k = h_k-1/2
        w = np.zeros(k + 1)
        w[:k] += 0.5 * h[:k]
        w[1:k + 1] += 0.5 * h[:k]
        acc = (w[:, None] ** 2 * var[:k + 1]).sum(axis=0)
        out[k] = np.sqrt(acc)
    return out


def entropy_scan(ctx, hop, layer, eps, eps_seed, U, mus, L_lo, L_hi, dtau, sites, n_warmup, n_measure, seed,
                 **kw):
    """Per-site entropy at the temperature between T_hi = 1/(L_lo dtau) and
    T_lo = 1/(L_hi dtau) on the grid mus (the first point taken as empty).
    Returns dict(s (len(mus), sites), s_err (statistical, from the last
    iteration's bins at every point), n_lo, n_hi, T_lo, T_hi, T, iterations,
    last_change (density_scan's, both temperatures), proposals)."""
    lat = hfqmc.Lattice(ctx, hop, layer)
    try:
        (n_lo, n_hi), (e_lo, e_hi), (it_lo, it_hi), props, (c_lo, c_hi) = density_scan(
            ctx, lat, hop, layer, eps, eps_seed, U, mus, (L_hi, L_lo), dtau, sites, n_warmup, n_measure,
            seed, **kw)
    finally:
        lat.close()
    T_lo, T_hi = 1.0 / (L_hi * dtau), 1.0 / (L_lo * dtau)
    s = hfqmc.entropy(mus, n_lo.sum(axis=2), n_hi.sum(axis=2), T_lo, T_hi)
    s_err = entropy_error(mus, e_lo, e_hi, T_lo, T_hi)
    return dict(s=s, s_err=s_err, n_lo=n_lo, n_hi=n_hi, T_lo=T_lo, T_hi=T_hi, T=0.5 * (T_lo + T_hi),
                iterations=it_lo + it_hi, last_change=np.concatenate([c_lo, c_hi]), proposals=props)


def find_mu(ctx, hop, layer, eps, U, L, dtau, sites, target, mu_lo, mu_hi, n_warmup, n_measure, seed, tol_n=0.5,
            max_steps=30, n_freq=500, tol=2e-3, max_iter=10, n_bins=16):
    """Chemical potential (Hartree-shifted) for which the converged lattice
    holds `target` atoms (n_up + n_dn summed over `sites`), by bisection on
    [mu_lo, mu_hi] (N grows with mu); each step is a converged RDMFT loop
    started from the nearest converged self-energy so far.  Returns
    dict(mu, atoms, steps: [(mu, atoms)])."""
    _check_seed_room(max_iter)
    lat = hfqmc.Lattice(ctx, hop, layer)
    N = lat.n_sites
    beta = L * dtau
    seen = []  # (mu, atoms, sigma)

    def atoms_at(mu):
        if seen:
            sigma0 = min(seen, key=lambda t: abs(t[0] - mu))[2]
        else:
            sigma0 = np.full((2, n_freq, N), -0.5 * U, dtype=np.complex128)
        r = RDMFT(ctx, hop, layer, eps, mu, U, beta, L, n_freq=n_freq, sigma0=sigma0, lattice=lat)
        out = r.converge(sites, n_warmup, n_measure, seed + SEED_STRIDE * len(seen), tol=tol, max_iter=max_iter, n_bins=n_bins)
        n = float(out["density"].sum())
        seen.append((mu, n, r.sigma.cpu().numpy()))
        r.close()
        return n

    try:
        lo, hi = mu_lo, mu_hi
        n_lo, n_hi = atoms_at(lo), atoms_at(hi)
        if not (n_lo <= target <= n_hi):
            raise ValueError(f"target {target} outside [{n_lo:.3f}, {n_hi:.3f}] on [{lo}, {hi}]")
        mu, n = (lo, n_lo) if abs(n_lo - target) < abs(n_hi - target) else (hi, n_hi)
        for _ in range(max_steps):
            if abs(n - target) < tol_n:
                break
            mid = 0.5 * (lo + hi)
            n_mid = atoms_at(mid)
            if n_mid < target:
                lo = mid
            else:
                hi = mid
            mu, n = mid, n_mid
    finally:
        lat.close()
    return dict(mu=mu, atoms=n, steps=[(m, a) for m, a, _ in seen])
