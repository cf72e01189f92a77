"""Seeded synthetic inputs: Weiss functions of trapped Hubbard lattices.

This module only *generates inputs*.  It holds none of the Hirsch-Fye method's
arithmetic and is the one module that both the HIP path's tests/benchmarks and
the CPU oracle read.

Every impurity problem is defined, as in the paper's real-space DMFT (Eq. (2)
and the local self-energy assumption after it), by the Weiss function of one
inequivalent lattice site.  The synthetic workloads take the non-interacting
(U = 0, Hartree-shifted) lattice of Eq. (1): the one-body matrix per spin is

    H^sigma = -t * adjacency + diag(V_i - mu_eff - sigma * h_i),
    V_i = V0 * r_i^2 (trap of Eq. (1), r in lattice units),
    mu_eff = mu - U/2 (the HS decoupling moves -U(n_up + n_dn)/2 into the
    one-body part), h_i = h * (-1)^(x+y) a staggered seed field,

and the Weiss samples of site i are

    g_i^sigma(tau_k) = sum_m phi_m(i)^2 exp(-e_m tau_k) / (1 + exp(-beta e_m)),
    tau_k = k * beta / L, k = 0..L-1   (k = 0 is tau = 0+).
"""
from __future__ import annotations

import numpy as np

# ----------------------------------------------------------------- lattices


def square_adjacency(nx: int, ny: int, periodic: bool = False) -> np.ndarray:
    N = nx * ny
    A = np.zeros((N, N))
    for x in range(nx):
        for y in range(ny):
            i = x * ny + y
            for dx, dy in ((1, 0), (0, 1)):
                xx, yy = x + dx, y + dy
                if periodic:
                    xx %= nx
                    yy %= ny
                elif xx >= nx or yy >= ny:
                    continue
                j = xx * ny + yy
                if j != i:
                    A[i, j] = A[j, i] = 1.0
    return A


def chain_adjacency(n: int) -> np.ndarray:
    A = np.zeros((n, n))
    for i in range(n - 1):
        A[i, i + 1] = A[i + 1, i] = 1.0
    return A


def trapped_square_onebody(nx, ny, V0, mu_eff, h=0.0, t=1.0):
    """(H_up, H_dn, coords) for an open nx x ny square lattice centred on a site."""
    A = square_adjacency(nx, ny)
    cx, cy = (nx - 1) / 2.0, (ny - 1) / 2.0
    coords = np.array([(x, y) for x in range(nx) for y in range(ny)])
    r2 = (coords[:, 0] - cx) ** 2 + (coords[:, 1] - cy) ** 2
    stag = np.where((coords.sum(axis=1) % 2) == 0, 1.0, -1.0)
    base = -t * A + np.diag(V0 * r2 - mu_eff)
    Hu = base + np.diag(-h * stag)
    Hd = base + np.diag(+h * stag)
    return Hu, Hd, coords


def _occ_weight(e, beta, taus):
    """exp(-e tau) (1 - f(e)), evaluated with non-positive exponents only."""
    e = e[None, :]
    t = taus[:, None]
    pos = e >= 0
    a = np.where(pos, np.exp(-np.where(pos, e, 0) * t) / (1.0 + np.exp(-beta * np.where(pos, e, 0))), 0.0)
    en = np.where(pos, 0, e)
    b = np.where(~pos, np.exp(en * (beta - t)) / (1.0 + np.exp(beta * en)), 0.0)
    return a + b  # (ntau, nmodes)


def weiss_from_onebody(H: np.ndarray, sites, beta: float, L: int) -> np.ndarray:
    """Weiss samples g_i(tau_k), k = 0..L-1, for each site in `sites`: (len(sites), L)."""
    e, phi = np.linalg.eigh(H)
    taus = np.arange(L) * (beta / L)
    W = _occ_weight(e, beta, taus)          # (L, M)
    P = phi[np.asarray(sites), :] ** 2      # (S, M)
    return P @ W.T


def densities_from_onebody(H: np.ndarray, beta: float) -> np.ndarray:
    """U = 0 occupation per site and spin: sum_m phi_m(i)^2 f(e_m)."""
    e, phi = np.linalg.eigh(H)
    f = 0.5 * (1.0 - np.tanh(0.5 * beta * e))
    return (phi ** 2) @ f


# ---------------------------------------------------------------- workloads


def _problem(L, beta, U, weiss, n_warmup, n_measure, seed, site, n_bins=32, recompute_every=50):
    return dict(L=int(L), beta=float(beta), U=float(U), weiss=np.ascontiguousarray(weiss, dtype=np.float64),
                n_warmup=int(n_warmup), n_measure=int(n_measure), recompute_every=int(recompute_every),
                n_bins=int(n_bins), seed=int(seed), site=int(site))


def plain_4x4(n_warmup=200, n_measure=2000, seed=1):
    """16 impurities: every site of an open 4x4 lattice, t = 1, mu_eff = 0
    (mu = U/2), U = 4, beta = 4, dtau = 0.25 (L = 16)."""
    U, beta, L = 4.0, 4.0, 16
    Hu, Hd, _ = trapped_square_onebody(4, 4, 0.0, 0.0)
    gu = weiss_from_onebody(Hu, range(16), beta, L)
    gd = weiss_from_onebody(Hd, range(16), beta, L)
    return [_problem(L, beta, U, np.stack([gu[i], gd[i]]), n_warmup, n_measure, seed, i) for i in range(16)]


def trapped_square(n, V0, U, beta, L, mu_eff, h, n_warmup, n_measure, seed, n_min=1e-3):
    """Occupied sites (U = 0 density n_up + n_dn > n_min) of an open n x n trapped lattice."""
    Hu, Hd, coords = trapped_square_onebody(n, n, V0, mu_eff, h)
    dens = densities_from_onebody(Hu, beta) + densities_from_onebody(Hd, beta)
    sites = np.nonzero(dens > n_min)[0]
    gu = weiss_from_onebody(Hu, sites, beta, L)
    gd = weiss_from_onebody(Hd, sites, beta, L)
    probs = [_problem(L, beta, U, np.stack([gu[k], gd[k]]), n_warmup, n_measure, seed, int(s))
             for k, s in enumerate(sites)]
    return probs, sites, coords


def trapped_lattice(n, V0, beta, mu_eff, h, n_min=1e-3):
    """Inputs of the lattice self-consistency for an open n x n trap, sites
    numbered row by row (rows are the layers): hop (N, N), eps (2, N) (trap
    potential -/+ the staggered seed field), and the sites with U = 0 density
    n_up + n_dn > n_min at inverse temperature beta (the ones solved; the same
    list as trapped_square)."""
    Hu, Hd, coords = trapped_square_onebody(n, n, V0, mu_eff, h)
    hop = Hu - np.diag(np.diag(Hu))
    eps = np.stack([np.diag(Hu), np.diag(Hd)]) + mu_eff
    dens = densities_from_onebody(Hu, beta) + densities_from_onebody(Hd, beta)
    return hop, eps, np.nonzero(dens > n_min)[0].astype(np.int32)


def trapped_21x21(n_warmup=1000, n_measure=10000, seed=2):
    """Trapped 2D cloud: 21x21, V0 = 0.05, U = 8, beta = 10, L = 40, mu = U/2, AF seed h = 0.1."""
    return trapped_square(21, 0.05, 8.0, 10.0, 40, 0.0, 0.1, n_warmup, n_measure, seed)[0]


C5_MU_EFF = 3.154


def slab_41x41(n_warmup=1000, n_measure=10000, seed=5, mu_eff=C5_MU_EFF):
    """Central slab: 41x41, V0 = 0.02, U = 8, beta = 16, dtau = 0.2 (L = 80), AF seed h = 0.1."""
    return trapped_square(41, 0.02, 8.0, 16.0, 80, mu_eff, 0.1, n_warmup, n_measure, seed)[0]


def chain_batch(n_imp=512, Ls=(32, 48, 64, 96, 128), beta=8.0, U_range=(4.0, 12.0), mu_range=(-1.0, 1.0),
                n_warmup=200, n_measure=2000, seed=3, chain_len=64):
    """Uneven-L batch: L ~ U(Ls), U ~ U(U_range), centre site of an open chain
    at mu_eff ~ U(mu_range), beta fixed (dtau = beta / L)."""
    rng = np.random.default_rng(seed)
    Lsel = rng.choice(np.asarray(Ls), size=n_imp)
    Us = rng.uniform(*U_range, size=n_imp)
    mus = rng.uniform(*mu_range, size=n_imp)
    A = chain_adjacency(chain_len)
    centre = chain_len // 2
    out = []
    for i in range(n_imp):
        H = -A - mus[i] * np.eye(chain_len)
        g = weiss_from_onebody(H, [centre], beta, int(Lsel[i]))[0]
        out.append(_problem(Lsel[i], beta, Us[i], np.stack([g, g]), n_warmup, n_measure, seed, i))
    return out


def chain_batch_L64(n_imp=512, n_warmup=200, n_measure=2000, seed=3):
    """The chain batch generator with every impurity at L = 64 (dtau = 0.125)."""
    return chain_batch(n_imp=n_imp, Ls=(64,), n_warmup=n_warmup, n_measure=n_measure, seed=seed)


def serving_requests(n_sites=200, n_iter=10, rate=200.0, Ls=(20, 40, 80, 160), weights=(4, 3, 2, 1),
                     U=8.0, dtau=0.25, sweeps=5000, seed=4, chain_len=64):
    """Poisson request stream: per site an L from Ls (weights), 10 simulated DMFT
    iterations; iteration j uses mu_eff + 0.02 j.  Returns (sites, arrivals) where
    sites[i] = dict(L, beta, U, mu_eff, seed) and arrivals are the first-iteration
    arrival times (later iterations arrive when the previous result returns)."""
    rng = np.random.default_rng(seed)
    p = np.asarray(weights, dtype=float) / np.sum(weights)
    Lsel = rng.choice(np.asarray(Ls), size=n_sites, p=p)
    mus = rng.uniform(-1.0, 1.0, size=n_sites)
    gaps = rng.exponential(1.0 / rate, size=n_sites)
    arrivals = np.cumsum(gaps)
    A = chain_adjacency(chain_len)
    centre = chain_len // 2
    sites = []
    for i in range(n_sites):
        L = int(Lsel[i])
        sites.append(dict(L=L, beta=L * dtau, U=U, mu_eff=float(mus[i]), seed=seed, site=i))

    def weiss(site, it):
        H = -A - (site["mu_eff"] + 0.02 * it) * np.eye(chain_len)
        g = weiss_from_onebody(H, [centre], site["beta"], site["L"])[0]
        return np.stack([g, g])

    return sites, arrivals, weiss


def atom_problem(L, beta, U, mu, h=0.0, n_warmup=200, n_measure=2000, seed=7, site=0, n_bins=32):
    """Isolated atom (no bath), Hartree-shifted levels -mu - sigma h + U/2."""
    taus = np.arange(L) * (beta / L)
    g = []
    for sigma in (+1, -1):
        e = -mu - sigma * h + 0.5 * U
        g.append(np.exp(-e * taus) / (1.0 + np.exp(-beta * e)))
    return _problem(L, beta, U, np.stack(g), n_warmup, n_measure, seed, site, n_bins=n_bins)


def two_site_problem(L, beta, U, mu, V, eb, h=0.0, n_warmup=200, n_measure=2000, seed=8, site=0, n_bins=32):
    """Impurity of a two-site Anderson model (bath level eb - mu, hybridisation V)."""
    out = []
    for sigma in (+1, -1):
        K = np.array([[-mu + 0.5 * U - sigma * h, V], [V, eb - mu]])
        out.append(weiss_from_onebody(K, [0], beta, L)[0])
    return _problem(L, beta, U, np.stack(out), n_warmup, n_measure, seed, site, n_bins=n_bins)
