"""Pins of the dtau -> 0 extrapolation oracle (CPU): exact polynomials are
recovered, error propagation matches the textbook straight-line formulas, and
exact discrete results of the two-site Anderson model (enumeration of every
field configuration at several L) extrapolate onto exact diagonalisation far
more closely than any single L comes."""
import numpy as np

import oracle
from oracle import exact as ex
from oracle import trotter as tr
from paper_1006_2716_amd import workloads as wl


def test_exact_polynomials_are_recovered():
    d = np.array([0.5, 0.4, 0.25, 0.2, 0.125])
    y = 0.3 - 1.7 * d ** 2 + 2.5 * d ** 4
    c, _ = tr.fit(d, y, order=2)
    assert np.allclose(c, [0.3, -1.7, 2.5], atol=1e-10)
    c1, _ = tr.fit(d[:2], 0.3 - 1.7 * d[:2] ** 2, order=1)
    assert np.allclose(c1, [0.3, -1.7], atol=1e-12)


def test_errors_follow_the_straight_line_formulas():
    """Weighted straight line in x = dtau^2: var(c0) = S_xx / D, var(c1) = S / D,
    D = S S_xx - S_x^2, with S = sum w, S_x = sum w x, S_xx = sum w x^2."""
    d = np.array([0.5, 0.35, 0.25, 0.125])
    e = np.array([0.01, 0.02, 0.015, 0.03])
    y = np.array([0.2, 0.25, 0.27, 0.3])
    c, ce = tr.fit(d, y, e, order=1)
    x, w = d ** 2, 1 / e ** 2
    S, Sx, Sxx, Sy, Sxy = w.sum(), (w * x).sum(), (w * x * x).sum(), (w * y).sum(), (w * x * y).sum()
    D = S * Sxx - Sx ** 2
    assert np.allclose(c, [(Sxx * Sy - Sx * Sxy) / D, (S * Sxy - Sx * Sy) / D], rtol=1e-12)
    assert np.allclose(ce, [np.sqrt(Sxx / D), np.sqrt(S / D)], rtol=1e-12)


def test_enumeration_extrapolates_onto_exact_diagonalisation():
    beta, U, mu, V, eb = 2.0, 4.0, 1.0, 0.8, 0.4
    ed = ex.ed_two_site(beta, U, mu, V, eb)
    Ls = [4, 6, 8, 10]
    vals = {k: [] for k in ("n_up", "docc")}
    for L in Ls:
        p = wl.two_site_problem(L, beta, U, mu, V, eb, h=0.0)
        v, _, _ = ex.enumerate_fields(p["weiss"][0], p["weiss"][1], oracle.lam(beta / L, U))
        vals["n_up"].append(v[2 * L + 2])
        vals["docc"].append(v[2 * L + 4])
    d = beta / np.array(Ls)
    for k in ("n_up", "docc"):
        single = abs(vals[k][-1] - ed[k])
        c2, _ = tr.fit(d, vals[k], order=2)
        assert abs(c2[0] - ed[k]) < single / 20, (k, single, c2[0] - ed[k])
        c1, _ = tr.fit(d[-2:], vals[k][-2:], order=1)
        assert abs(c1[0] - ed[k]) < single / 3, (k, single, c1[0] - ed[k])
