"""Plain reference for the real-space DMFT self-consistency around the solver.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): used by ``tests/``
and nothing in the product package.  Dense numpy, complex128, no blocking:
every function is its defining formula written out.

Conventions (shared with the solver's inputs).  Site i, spin s (0 = up,
1 = down), one-body matrix H_s = hop + diag(eps_s) (hop real symmetric, eps
the trap potential plus any seed field), chemical potential ``mu`` of the
Hartree-shifted levels (mu - U/2 in the paper's notation) and the self-energy
``sigma`` relative to those levels (Sigma - U/2).  The solver's Weiss samples
are g(tau) = <c(tau) c^+> = -G(tau) on tau_l = l beta / L.  Matsubara
frequencies w_n = (2n + 1) pi / beta, n = 0 .. n_freq - 1; negative ones follow
from G(-iw) = conj G(iw).

What the paper fixes: the lattice Dyson equation, Eq. (2), with a site-diagonal
self-energy (the sentence after it), solved frequency by frequency.  What it
leaves to the solver literature (readings, stated where used):
  * the impurity Dyson equation  Weiss^-1 = G_loc^-1 + sigma;
  * iw -> tau: the exact transform of 1 / (iw - e) with e the Weiss
    function's site level, plus the truncated Matsubara sum of the rest;
  * tau -> iw: the Hartree-corrected Weiss function plus the exact transform of
    the piecewise-linear interpolant of (g_imp - g_Hartree) on the L + 1 grid;
  * the self-energy from those transforms below w_n dtau = pi / 2 (n < L / 4),
    above it the first two terms of its large-frequency expansion.
"""
from __future__ import annotations

import numpy as np


def matsubara(beta: float, n_freq: int) -> np.ndarray:
    """Fermionic Matsubara frequencies (2n + 1) pi T, n = 0 .. n_freq - 1 (the
    grid stated with Eq. (2))."""
    return (2.0 * np.arange(n_freq) + 1.0) * np.pi / beta


def lattice_local_green(hop, eps, mu, sigma, beta, n_index=None):
    """Eq. (2): G(iw_n) = [(iw_n + mu) 1 - hop - diag(eps_s) - diag(sigma_s(iw_n))]^-1,
    one dense inverse per spin and frequency; returns the site-diagonal part.

    hop (N, N) real, eps (2, N) real, sigma (2, K, N) complex at the Matsubara
    indices n_index (default 0 .. K - 1).  Returns G_loc (2, K, N) complex."""
    hop = np.asarray(hop, dtype=np.float64)
    N = hop.shape[0]
    K = sigma.shape[1]
    idx = np.arange(K) if n_index is None else np.asarray(n_index)
    w = (2.0 * idx + 1.0) * np.pi / beta
    out = np.zeros((2, K, N), dtype=np.complex128)
    for s in range(2):
        for k in range(K):
            A = (1j * w[k] + mu) * np.eye(N) - hop - np.diag(eps[s]) - np.diag(sigma[s, k])
            out[s, k] = np.diag(np.linalg.inv(A))
    return out


def weiss_iw(gloc, sigma):
    """Impurity Dyson equation (reading): Weiss(iw)^-1 = G_loc(iw)^-1 + sigma(iw)."""
    return 1.0 / (1.0 / gloc + sigma)


def model_tau(e, beta, taus):
    """g(tau) of a single level e, the transform of 1 / (iw - e):
    exp(-e tau) / (1 + exp(-beta e)) for 0 <= tau <= beta, evaluated with
    non-positive exponents only."""
    e = float(e)
    taus = np.asarray(taus, dtype=np.float64)
    if e >= 0:
        return np.exp(-e * taus) / (1.0 + np.exp(-beta * e))
    return np.exp(e * (beta - taus)) / (np.exp(beta * e) + 1.0)


def tau_from_iw(giw, e, beta, taus):
    """g(tau) = -T sum_{n in Z} exp(-iw_n tau) G(iw_n), split into the level
    1 / (iw - e), transformed exactly, and the rest, summed over the kept
    frequencies and their negatives (reading: the tail is the Weiss
    function's own level, so the remainder falls off like 1 / w^3).
    giw (n_freq,) complex.  taus in [0, beta]; tau = 0 means 0+, beta means beta-."""
    giw = np.asarray(giw, dtype=np.complex128)
    w = matsubara(beta, giw.size)
    rest = giw - 1.0 / (1j * w - e)
    taus = np.asarray(taus, dtype=np.float64)
    out = model_tau(e, beta, taus)
    for k, t in enumerate(taus):
        out[k] -= (2.0 / beta) * np.sum((np.exp(-1j * w * t) * rest).real)
    return out


def iw_from_linear_tau(d, beta, n_freq):
    """Integral over [0, beta] of exp(iw_n tau) d_lin(tau), d_lin the
    piecewise-linear interpolant of d on tau_k = k beta / L, k = 0 .. L
    (d has L + 1 samples).  Written segment by segment: on [a, a + h] with end
    values p, q the integrand is (p + (q - p)(tau - a)/h) exp(iw tau), whose
    integral is exact in closed form."""
    d = np.asarray(d, dtype=np.float64)
    L = d.size - 1
    h = beta / L
    w = matsubara(beta, n_freq)
    out = np.zeros(n_freq, dtype=np.complex128)
    for n in range(n_freq):
        x = 1j * w[n]
        for k in range(L):
            a = k * h
            p, q = d[k], d[k + 1]
            # int_0^h exp(x s) ds and int_0^h s exp(x s) ds
            i0 = (np.exp(x * h) - 1.0) / x
            i1 = h * np.exp(x * h) / x - (np.exp(x * h) - 1.0) / (x * x)
            out[n] += np.exp(x * a) * (p * i0 + (q - p) / h * i1)
    return out


def sigma_cutoff(L: int) -> int:
    """Frequencies n < L / 4 (w_n dtau < pi / 2) take the self-energy from the
    sampled g(tau); the piecewise-linear transform loses accuracy towards the
    grid's Nyquist frequency pi / dtau."""
    return max(1, L // 4)


def sigma_update(weiss, e, gimp_tau, n_other, U, beta):
    """New self-energy of one site and spin from the solver's result.

    weiss (n_freq,) the Weiss function the solver was given, e its level,
    gimp_tau (L + 1,) the solver's g(tau_k), n_other the solver's density of
    the other spin.  Reading: the Hartree term sigma_inf = U (n_other - 1/2) is
    the exact large-w limit of sigma; the Weiss function shifted by it,
    W_H = 1 / (Weiss^-1 - sigma_inf), is transformed exactly (level e +
    sigma_inf plus the Matsubara rest) and only the difference to it is
    interpolated; sigma(iw_n) = Weiss^-1 - G_imp^-1 for n < sigma_cutoff(L),
    sigma_inf + U^2 n_other (1 - n_other) / (iw_n) above (the exact first two
    moments of the self-energy of the Hubbard interaction)."""
    weiss = np.asarray(weiss, dtype=np.complex128)
    nf = weiss.size
    L = len(gimp_tau) - 1
    s_inf = U * (n_other - 0.5)
    wh = 1.0 / (1.0 / weiss - s_inf)
    taus = np.arange(L + 1) * (beta / L)
    g_h = tau_from_iw(wh, e + s_inf, beta, taus)
    # G = -int exp(iw tau) g(tau) dtau, with the Hartree part exact
    g_imp = wh - iw_from_linear_tau(np.asarray(gimp_tau) - g_h, beta, nf)
    sig = 1.0 / weiss - 1.0 / g_imp
    nc = sigma_cutoff(L)
    w = matsubara(beta, nf)
    sig[nc:] = s_inf + U * U * n_other * (1.0 - n_other) / (1j * w[nc:])
    return sig
