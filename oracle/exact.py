"""Exact results that the Hirsch-Fye Markov chain must reproduce.

TEST INFRASTRUCTURE ONLY (part of the oracle; see ``oracle/__init__.py``).

Everything here is written with numpy/scipy library primitives (det, solve,
expm, eigh) and shares no code with the C chain in ``hfqmc_ref.c``, so the two
cross-check each other:

* ``enumerate_fields`` -- the discrete (Trotterised) impurity problem summed
  over all 2^L Ising fields with weight w(s) = prod_sigma det M_sigma(s)
  (Hirsch-Fye weights of the solver named in "Model and Methods").
* ``atom_exact`` -- the isolated atom in closed form.  Its one-body and U terms
  commute, so the discrete problem is exact at every L.
* ``bss_green_diag`` / ``bss_weight`` -- the determinantal (BSS) form of the
  same discrete problem on an explicit impurity+bath one-body matrix K, with
  B_l = exp(V_l) exp(-dtau K) and the equal-time impurity Green function
  (1 + B_l ... B_1 B_L ... B_{l+1})^{-1}_{00}.
* ``ed_two_site`` -- exact diagonalisation of the continuous-time two-site
  Anderson model; the discrete problem converges to it as O(dtau^2).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sla


def lam_exact(dtau: float, U: float) -> float:
    """Root of cosh(lambda) = exp(dtau U / 2), by numpy's arccosh."""
    return float(np.arccosh(np.exp(0.5 * dtau * U)))


def weiss_matrix_np(g: np.ndarray) -> np.ndarray:
    """Antiperiodic L x L matrix from the samples g(tau_k), k = 0..L-1."""
    L = len(g)
    i = np.arange(L)[:, None]
    j = np.arange(L)[None, :]
    d = i - j
    return np.where(d >= 0, g[np.mod(d, L)], -g[np.mod(d, L)])


def estimators(Gu: np.ndarray, Gd: np.ndarray):
    """Per-configuration estimators: g_up(0..L), g_dn(0..L), n_up, n_dn, d.

    g(tau_k) is the antiperiodic average over the k-th (wrapped) diagonal.
    """
    L = Gu.shape[0]
    out = []
    for G in (Gu, Gd):
        g = np.empty(L + 1)
        for k in range(L):
            acc = 0.0
            for l in range(L):
                i = l + k
                acc += G[i, l] if i < L else -G[i - L, l]
            g[k] = acc / L
        g[L] = 1.0 - np.trace(G) / L
        out.append(g)
    nu = 1.0 - np.trace(Gu) / L
    nd = 1.0 - np.trace(Gd) / L
    d = np.mean((1.0 - np.diag(Gu)) * (1.0 - np.diag(Gd)))
    return np.concatenate([out[0], out[1], [nu, nd, d]])


def hs_matrix(g: np.ndarray, lam: float, sigma: int, s: np.ndarray) -> np.ndarray:
    """M_sigma(s) = 1 + (1 - G0)(exp(V_sigma) - 1)."""
    L = len(g)
    G0 = weiss_matrix_np(g)
    E = np.diag(np.exp(sigma * lam * np.asarray(s, dtype=float)) - 1.0)
    return np.eye(L) + (np.eye(L) - G0) @ E


def green_np(g: np.ndarray, lam: float, sigma: int, s: np.ndarray) -> np.ndarray:
    """G_sigma(s) = M_sigma(s)^{-1} G0 via numpy.linalg.solve."""
    return np.linalg.solve(hs_matrix(g, lam, sigma, s), weiss_matrix_np(g))


def enumerate_fields(g_up: np.ndarray, g_dn: np.ndarray, lam: float):
    """Exact expectation of the estimators over all 2^L fields.

    Returns (mean_values, weights, configs) where weights are normalised."""
    L = len(g_up)
    configs = np.array(list(itertools.product([1, -1], repeat=L)), dtype=np.int8)
    w = np.empty(len(configs))
    vals = np.empty((len(configs), 2 * (L + 1) + 3))
    for c, s in enumerate(configs):
        Mu = hs_matrix(g_up, lam, +1, s)
        Md = hs_matrix(g_dn, lam, -1, s)
        w[c] = np.linalg.det(Mu) * np.linalg.det(Md)
        Gu = np.linalg.solve(Mu, weiss_matrix_np(g_up))
        Gd = np.linalg.solve(Md, weiss_matrix_np(g_dn))
        vals[c] = estimators(Gu, Gd)
    wn = w / w.sum()
    return wn @ vals, wn, configs


def free_green_tau(K: np.ndarray, site: int, beta: float, taus: np.ndarray) -> np.ndarray:
    """g(tau) = sum_m phi_m(site)^2 exp(-e_m tau) / (1 + exp(-beta e_m))."""
    e, phi = np.linalg.eigh(K)
    w = phi[site] ** 2
    out = np.empty(len(taus))
    for k, t in enumerate(taus):
        out[k] = np.sum(w * np.exp(-e * t) / (1.0 + np.exp(-beta * e)))
    return out


def atom_exact(beta: float, U: float, mu: float, h: float = 0.0, taus=None):
    """Closed forms for one isolated site with levels eps_sigma = -mu - sigma h.

    Returns dict with n_up, n_dn, docc and (if taus given) g_up(tau), g_dn(tau).
    """
    eu, ed = -mu - h, -mu + h
    a = np.exp(-beta * eu)
    b = np.exp(-beta * ed)
    c = np.exp(-beta * (eu + ed + U))
    Z = 1.0 + a + b + c
    res = dict(n_up=(a + c) / Z, n_dn=(b + c) / Z, docc=c / Z)
    if taus is not None:
        t = np.asarray(taus, dtype=float)
        res["g_up"] = (np.exp(-t * eu) + b * np.exp(-t * (eu + U))) / Z
        res["g_dn"] = (np.exp(-t * ed) + a * np.exp(-t * (ed + U))) / Z
    return res


def atom_weiss(beta: float, U: float, mu: float, h: float, L: int):
    """Hartree-shifted Weiss samples of the isolated atom: level eps_sigma + U/2."""
    taus = np.arange(L) * (beta / L)
    out = []
    for sigma in (+1, -1):
        e = -mu - sigma * h + 0.5 * U
        out.append(np.exp(-e * taus) / (1.0 + np.exp(-beta * e)))
    return np.array(out)


def bss_products(K: np.ndarray, lam: float, sigma: int, s: np.ndarray, beta: float):
    L = len(s)
    dt = beta / L
    Bk = sla.expm(-dt * K)
    N = K.shape[0]
    Bs = []
    for l in range(L):
        v = np.ones(N)
        v[0] = np.exp(sigma * lam * s[l])
        Bs.append(np.diag(v) @ Bk)
    return Bs


def bss_green_diag(K: np.ndarray, lam: float, sigma: int, s: np.ndarray, beta: float) -> np.ndarray:
    """Impurity element of (1 + B_l ... B_1 B_L ... B_{l+1})^{-1} for each slice l."""
    L = len(s)
    Bs = bss_products(K, lam, sigma, s, beta)
    N = K.shape[0]
    out = np.empty(L)
    for l in range(L):
        P = np.eye(N)
        for m in list(range(l + 1, L)) + list(range(0, l + 1)):
            P = Bs[m] @ P
        out[l] = np.linalg.inv(np.eye(N) + P)[0, 0]
    return out


def bss_green_full(K: np.ndarray, lam: float, sigma: int, s: np.ndarray, beta: float) -> np.ndarray:
    """Full L x L impurity Green matrix from the BSS products.

    With G_l the equal-time matrix at slice l and B(l, l') = B_l ... B_{l'+1}:
    X[l, l'] = [B(l, l') G_l']_00 for l >= l', and -[(1 - G_l) B(l', l)^{-1}]_00
    for l < l'.  The Hirsch-Fye matrix M^{-1} G0 is the same object in the gauge
    exp(-V) X exp(V) (identical diagonal)."""
    L = len(s)
    Bs = bss_products(K, lam, sigma, s, beta)
    N = K.shape[0]
    I = np.eye(N)

    def prod(a, b):  # B_b ... B_a
        P = np.eye(N)
        for m in range(a, b + 1):
            P = Bs[m] @ P
        return P

    Geq = []
    for l in range(L):
        P = np.eye(N)
        for m in list(range(l + 1, L)) + list(range(0, l + 1)):
            P = Bs[m] @ P
        Geq.append(np.linalg.inv(I + P))
    X = np.empty((L, L))
    for l in range(L):
        for lp in range(L):
            if l >= lp:
                X[l, lp] = (prod(lp + 1, l) @ Geq[lp])[0, 0]
            else:
                X[l, lp] = -((I - Geq[l]) @ np.linalg.inv(prod(l + 1, lp)))[0, 0]
    v = np.exp(sigma * lam * np.asarray(s, dtype=float))
    return (X / v[:, None]) * v[None, :]


def bss_weight(K: np.ndarray, lam: float, sigma: int, s: np.ndarray, beta: float) -> float:
    """det(1 + B_L ... B_1) for one spin."""
    Bs = bss_products(K, lam, sigma, s, beta)
    P = np.eye(K.shape[0])
    for B in Bs:
        P = B @ P
    return float(np.linalg.det(np.eye(K.shape[0]) + P))


def ed_two_site(beta: float, U: float, mu: float, V: float, eb: float):
    """Exact diagonalisation of the two-site Anderson model.

    H = sum_sigma [-mu n_d + (eb - mu) n_b + V (d^dag b + b^dag d)] + U n_d_up n_d_dn.
    Returns dict(n_up, n_dn, docc) of the impurity orbital.
    """
    # modes: 0 d_up, 1 d_dn, 2 b_up, 3 b_dn ; Jordan-Wigner on 16 states
    nm = 4
    dim = 1 << nm

    def ann(m):
        A = np.zeros((dim, dim))
        for st in range(dim):
            if st >> m & 1:
                sign = (-1) ** bin(st & ((1 << m) - 1)).count("1")
                A[st ^ (1 << m), st] = sign
        return A

    a = [ann(m) for m in range(nm)]
    n = [x.T @ x for x in a]
    H = -mu * (n[0] + n[1]) + (eb - mu) * (n[2] + n[3]) + U * n[0] @ n[1]
    for d, b in ((0, 2), (1, 3)):
        H += V * (a[d].T @ a[b] + a[b].T @ a[d])
    e, v = np.linalg.eigh(H)
    w = np.exp(-beta * (e - e.min()))
    Z = w.sum()

    def ev(O):
        return float(np.sum(w * np.einsum("ij,jk,ki->i", v.T, O, v)) / Z)

    return dict(n_up=ev(n[0]), n_dn=ev(n[1]), docc=ev(n[0] @ n[1]))
