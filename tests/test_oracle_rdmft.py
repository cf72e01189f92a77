"""Pins of the RDMFT oracle (CPU): each check compares against something other
than the oracle's own formula -- eigen-decompositions, closed-form integrals,
the isolated atom -- so that a dropped term, a wrong sign or a transposed
operand fails one of them."""
import numpy as np
import pytest

from oracle import exact as ex
from oracle import rdmft as rd
from paper_1006_2716_amd import workloads as wl


def _trap(nx, ny, V0=0.3, mu_eff=0.4, h=0.15):
    Hu, Hd, coords = wl.trapped_square_onebody(nx, ny, V0, mu_eff, h)
    hop = Hu - np.diag(np.diag(Hu))
    # site energies relative to mu: Hu = hop + diag(eps_up) - mu
    eps = np.stack([np.diag(Hu), np.diag(Hd)]) + mu_eff
    return hop, eps, mu_eff, (Hu, Hd)


def test_local_green_matches_eigen_decomposition():
    """Site-independent sigma = c: G_ii = sum_m phi_m(i)^2 / (iw + mu - E_m - c)."""
    hop, eps, mu, _ = _trap(4, 5)
    beta, nf = 3.0, 7
    c = np.array([0.2 - 0.3j, -0.1 - 0.05j])
    sigma = np.broadcast_to(c[:, None, None], (2, nf, 20)).copy()
    G = rd.lattice_local_green(hop, eps, mu, sigma, beta)
    w = rd.matsubara(beta, nf)
    for s in range(2):
        E, phi = np.linalg.eigh(hop + np.diag(eps[s]))
        for n in range(nf):
            ref = (phi ** 2) @ (1.0 / (1j * w[n] + mu - E - c[s]))
            assert np.max(np.abs(G[s, n] - ref)) < 1e-13


def test_local_green_at_selected_frequencies():
    hop, eps, mu, _ = _trap(3, 4)
    beta, nf = 2.0, 9
    sig = np.full((2, nf, 12), 0.1 - 0.2j)
    full = rd.lattice_local_green(hop, eps, mu, sig, beta)
    idx = [2, 7]
    part = rd.lattice_local_green(hop, eps, mu, sig[:, idx], beta, n_index=idx)
    assert np.array_equal(part, full[:, idx])


def test_local_green_without_hopping_is_the_site_resolvent():
    rng = np.random.default_rng(1)
    N, beta, nf = 6, 5.0, 4
    eps = rng.normal(size=(2, N))
    sig = rng.normal(size=(2, nf, N)) - 1j * rng.uniform(0.1, 1, size=(2, nf, N))
    G = rd.lattice_local_green(np.zeros((N, N)), eps, 0.3, sig, beta)
    w = rd.matsubara(beta, nf)
    ref = 1.0 / (1j * w[None, :, None] + 0.3 - eps[:, None, :] - sig)
    assert np.max(np.abs(G - ref)) < 1e-14


def test_single_level_transform_is_exact():
    beta, e = 4.0, -0.7
    w = rd.matsubara(beta, 50)
    taus = np.linspace(0, beta, 9)
    g = rd.tau_from_iw(1.0 / (1j * w - e), e, beta, taus)
    assert np.allclose(g, np.exp(-e * taus) / (1 + np.exp(-beta * e)), atol=1e-14)


@pytest.mark.parametrize("nf", [250, 500])
def test_local_weiss_tau_matches_eigen_form(nf):
    """sigma = 0: the Weiss function is the U = 0 lattice G_ii; its tau samples
    from the Matsubara sum must match the eigen-decomposition form, with the
    truncation error falling like 1 / n_freq^2."""
    hop, eps, mu, (Hu, Hd) = _trap(3, 4)
    beta, L = 4.0, 16
    G = rd.lattice_local_green(hop, eps, mu, np.zeros((2, nf, 12), complex), beta)
    taus = np.arange(L + 1) * (beta / L)
    errs = []
    for s, H in ((0, Hu), (1, Hd)):
        for i in (0, 5, 11):
            g = rd.tau_from_iw(G[s, :, i], eps[s, i] - mu, beta, taus)
            ref = ex.free_green_tau(H, i, beta, taus)
            ref[-1] = 1.0 - ref[0]  # tau = beta means beta-
            errs.append(np.max(np.abs(g - ref)))
            assert abs(g[0] + g[-1] - 1.0) < 1e-12
    err = max(errs)
    bound = {250: 2e-5, 500: 5e-6}[nf]
    assert err < bound, err


def test_linear_interpolant_transform_closed_forms():
    beta, L, nf = 2.5, 10, 6
    w = rd.matsubara(beta, nf)
    x = 1j * w
    taus = np.arange(L + 1) * (beta / L)
    a, b = 0.7, -0.4
    got = rd.iw_from_linear_tau(a + b * taus, beta, nf)
    # int_0^beta (a + b tau) exp(x tau) dtau with exp(x beta) = -1
    ref = -2 * a / x + b * (-beta / x + 2 / x ** 2)
    assert np.max(np.abs(got - ref)) < 1e-13


def test_linear_interpolant_transform_converges_like_dtau_squared():
    beta, e, nf = 3.0, 0.4, 4
    w = rd.matsubara(beta, nf)
    exact = -1.0 / (1j * w - e)  # int exp(iw tau) g(tau) for g of a single level
    errs = []
    for L in (16, 32, 64):
        taus = np.arange(L + 1) * (beta / L)
        errs.append(np.max(np.abs(rd.iw_from_linear_tau(rd.model_tau(e, beta, taus), beta, nf) - exact)))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_sigma_vanishes_at_U0_and_is_hartree_for_a_hartree_solver():
    hop, eps, mu, _ = _trap(3, 3)
    beta, L, nf = 4.0, 20, 200
    G = rd.lattice_local_green(hop, eps, mu, np.zeros((2, nf, 9), complex), beta)
    weiss = rd.weiss_iw(G[0, :, 4], np.zeros(nf))
    e = eps[0, 4] - mu
    taus = np.arange(L + 1) * (beta / L)
    g0 = rd.tau_from_iw(weiss, e, beta, taus)
    assert np.max(np.abs(rd.sigma_update(weiss, e, g0, 0.37, 0.0, beta))) < 1e-12
    # a solver that returns the Hartree-shifted Weiss function gives sigma = U (n - 1/2)
    # below the cutoff, and the two-moment tail above it
    U, n = 3.0, 0.37
    wh = 1.0 / (1.0 / weiss - U * (n - 0.5))
    gh = rd.tau_from_iw(wh, e + U * (n - 0.5), beta, taus)
    sig = rd.sigma_update(weiss, e, gh, n, U, beta)
    nc = rd.sigma_cutoff(L)
    assert nc == 5
    assert np.max(np.abs(sig[:nc] - U * (n - 0.5))) < 1e-10
    w = rd.matsubara(beta, nf)
    assert np.max(np.abs(sig[nc:] - U * (n - 0.5) + 1j * U * U * n * (1 - n) / w[nc:])) < 1e-13


def test_sigma_of_the_atom_converges_to_the_closed_form():
    """Isolated atom: Weiss = 1/(iw - e), exact g(tau) on the L + 1 grid; the
    self-energy from the transforms approaches the atomic one
    (iw - e) - G^-1 with G = (1 - n')/(iw - eps) + n'/(iw - eps - U), the
    error falling like dtau^2 at fixed low frequencies."""
    beta, U, mu, h, nf = 4.0, 3.0, 1.1, 0.2, 500
    at = ex.atom_exact(beta, U, mu, h)
    eps_up = -mu - h
    e = eps_up + 0.5 * U  # Hartree-shifted level the solver is given
    w = rd.matsubara(beta, nf)
    weiss = 1.0 / (1j * w - e)
    G = (1 - at["n_dn"]) / (1j * w - eps_up) + at["n_dn"] / (1j * w - eps_up - U)
    exact = (1j * w - e) - 1.0 / G
    errs = []
    for L in (32, 64, 128):
        taus = np.arange(L + 1) * (beta / L)
        g = ex.atom_exact(beta, U, mu, h, taus)["g_up"]
        sig = rd.sigma_update(weiss, e, g, at["n_dn"], U, beta)
        errs.append(np.max(np.abs(sig[:4] - exact[:4])))
        # above the cutoff: within the third moment's size of the exact atom
        nc = rd.sigma_cutoff(L)
        assert np.max(np.abs(sig[nc:] - exact[nc:]) * w[nc:] ** 2) < 3 * U ** 3
    assert errs[-1] < 2e-3
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_weiss_of_isolated_sites_is_the_bare_level_for_any_sigma():
    """Without hopping G_loc = 1 / (iw + mu - eps - sigma), so the impurity
    Dyson equation must give back 1 / (iw + mu - eps) whatever sigma is; a
    sign slip (G^-1 - sigma) leaves 2 sigma behind."""
    rng = np.random.default_rng(7)
    N, beta, nf, mu = 5, 3.0, 6, 0.25
    eps = rng.normal(size=(2, N))
    sig = rng.normal(size=(2, nf, N)) - 1j * rng.uniform(0.2, 2.0, size=(2, nf, N))
    gl = rd.lattice_local_green(np.zeros((N, N)), eps, mu, sig, beta)
    w = rd.matsubara(beta, nf)
    ref = 1.0 / (1j * w[None, :, None] + mu - eps[:, None, :])
    assert np.max(np.abs(rd.weiss_iw(gl, sig) - ref)) < 1e-13


def test_weiss_of_a_dimer_is_the_cavity_function():
    """Two sites joined by hopping t: the 2x2 inverse gives
    G_11 = z2 / (z1 z2 - t^2), z_i = iw + mu - eps_i - sigma_i, so the Weiss
    function of site 1 is 1 / (iw + mu - eps_1 - t^2 / z2): the cavity
    (hybridisation) form, independent of sigma_1 and depending on sigma_2."""
    t, mu, beta, nf = 0.8, 0.1, 4.0, 5
    eps = np.array([[0.3, -0.4], [0.5, 0.2]])
    rng = np.random.default_rng(3)
    sig = rng.normal(size=(2, nf, 2)) - 1j * rng.uniform(0.1, 1.5, size=(2, nf, 2))
    hop = np.array([[0.0, -t], [-t, 0.0]])
    gl = rd.lattice_local_green(hop, eps, mu, sig, beta)
    wf = rd.weiss_iw(gl, sig)
    iw = 1j * rd.matsubara(beta, nf)
    for s in range(2):
        z = iw[:, None] + mu - eps[s][None, :] - sig[s]
        ref0 = 1.0 / (iw + mu - eps[s, 0] - t * t / z[:, 1])
        ref1 = 1.0 / (iw + mu - eps[s, 1] - t * t / z[:, 0])
        assert np.max(np.abs(wf[s, :, 0] - ref0)) < 1e-13
        assert np.max(np.abs(wf[s, :, 1] - ref1)) < 1e-13
