"""Pins of the entropy oracle (CPU) against closed forms: free fermions on a
trapped lattice (total and per-site entropy from the eigen-decomposition) and
the isolated Hubbard atom (ln Z + (E - mu N) / T)."""
import numpy as np

from oracle import exact as ex
from oracle import thermo as th
from paper_1006_2716_amd import workloads as wl


def _fermi(x):
    return 0.5 * (1.0 - np.tanh(0.5 * x))


def _s_of_f(f):
    f = np.clip(f, 1e-300, 1 - 1e-16)
    return -(f * np.log(f) + (1 - f) * np.log1p(-f))


def test_free_fermions_total_and_local():
    Hu, _, _ = wl.trapped_square_onebody(5, 5, 0.3, 0.0, 0.0)
    E, phi = np.linalg.eigh(Hu)
    T, dT = 0.3, 0.003
    mu = np.linspace(E.min() - 12.0, 1.0, 1201)

    def dens(T_):
        return np.stack([(phi ** 2) @ _fermi((E - m) / T_) for m in mu])  # (K, sites)

    s = th.entropy_from_densities(mu, dens(T - dT), dens(T + dT), T - dT, T + dT)
    exact_local = np.stack([(phi ** 2) @ _s_of_f(_fermi((E - m) / T)) for m in mu])
    assert np.max(np.abs(s - exact_local)) < 2e-4
    assert abs(s[-1].sum() - exact_local[-1].sum()) < 2e-3


def test_hubbard_atom():
    U, T, dT = 4.0, 0.5, 0.005
    mu = np.linspace(-10.0, 3.0, 2601)

    def dens(T_):
        return np.array([[ex.atom_exact(1.0 / T_, U, m)["n_up"] * 2] for m in mu])

    s = th.entropy_from_densities(mu, dens(T - dT), dens(T + dT), T - dT, T + dT)[:, 0]
    b = 1.0 / T
    for k in (600, 1300, 2000, 2600):
        m = mu[k]
        w = np.array([1.0, np.exp(b * m), np.exp(b * m), np.exp(-b * (U - 2 * m))])  # 0, up, dn, both
        Z = w.sum()
        E = (w[3] * U) / Z
        N = (w[1] + w[2] + 2 * w[3]) / Z
        exact = np.log(Z) + b * (E - m * N)
        assert abs(s[k] - exact) < 2e-4, (m, s[k], exact)


def test_staggered_sign_pattern():
    coords = np.array([(0, 0), (0, 1), (1, 1), (2, 1)])
    assert np.array_equal(th.staggered([1.0, 1.0, 1.0, 1.0], coords), [1.0, -1.0, 1.0, -1.0])


def test_package_staggered_magnetization_matches_the_oracle():
    from paper_1006_2716_amd.thermo import staggered_magnetization
    rng = np.random.default_rng(2)
    _, _, coords = wl.trapped_square_onebody(5, 5, 0.1, 0.0)
    d = rng.uniform(0, 1, size=(25, 2))
    assert np.array_equal(staggered_magnetization(d, coords), th.staggered(d[:, 0] - d[:, 1], coords))


def test_entropy_error_propagation_matches_monte_carlo():
    """The propagated error of the trapezoid integral against the spread of
    the integral over many noisy copies of the same densities."""
    from paper_1006_2716_amd.thermo import entropy_error
    rng = np.random.default_rng(9)
    mu = np.sort(rng.uniform(-3, 1, size=12))
    n = rng.uniform(0, 1, size=(12, 3))
    e_lo, e_hi = rng.uniform(1e-3, 3e-3, size=(2, 12, 3))
    draws = [th.entropy_from_densities(mu, n + e_lo * rng.normal(size=n.shape), n + 0.01 + e_hi * rng.normal(
        size=n.shape), 0.2, 0.21)[-1] for _ in range(4000)]
    spread = np.std(draws, axis=0)
    assert np.allclose(entropy_error(mu, e_lo, e_hi, 0.2, 0.21)[-1], spread, rtol=0.06)
