"""The multiple-comparison rule used by the GPU statistics tests, checked on
synthetic bin series where the truth is known: agreeing chains pass, a
shifted observable or underestimated errors fail, the chance bound matches
the binomial distribution, and the binning analysis sees correlated bins."""
import numpy as np
import pytest

import stats_rule


def _fake(n_imp, nb, L, rng, shift=0.0, rho=0.0, symmetric=False):
    """Problem and result dicts whose bins hold AR(1) series of n_up, n_dn, d."""
    probs, a, b = [], [], []
    NV = 2 * (L + 1) + 3
    for _ in range(n_imp):
        w = np.ones((2, L)) if symmetric else np.stack([np.ones(L), 2 * np.ones(L)])
        probs.append(dict(L=L, weiss=w))
        for out, sh in ((a, shift), (b, 0.0)):
            bins = np.zeros((nb, NV))
            for col in range(2 * L + 2, 2 * L + 5):
                e = rng.normal(size=nb)
                x = np.empty(nb)
                x[0] = e[0] / np.sqrt(1 - rho ** 2)
                for i in range(1, nb):
                    x[i] = rho * x[i - 1] + e[i]
                bins[:, col] = 0.5 + 0.01 * x + (sh * 0.01 / np.sqrt(nb) if col == 2 * L + 4 else 0.0)
            out.append(dict(bins=bins))
    return probs, a, b


def test_agreeing_chains_pass():
    rng = np.random.default_rng(5)
    probs, a, b = _fake(256, 64, 8, rng)
    stats_rule.check(probs, a, b, "iid")
    probs, a, b = _fake(256, 64, 8, rng, rho=0.3)  # correlated bins: the binning analysis widens the errors
    stats_rule.check(probs, a, b, "ar1")


def test_shifted_observable_fails():
    rng = np.random.default_rng(6)
    probs, a, b = _fake(256, 64, 8, rng, shift=2.0)  # d shifted by 2 standard errors of one side
    with pytest.raises(AssertionError):
        stats_rule.check(probs, a, b, "shift")


def test_offsets_beyond_the_errors_fail():
    rng = np.random.default_rng(7)
    probs, a, b = _fake(256, 64, 8, rng)
    for r in a:  # every impurity off by 4 standard errors of one side, random sign
        r["bins"][:, 2 * 8 + 4] += 4 * 0.01 / np.sqrt(64) * rng.choice([-1.0, 1.0])
    with pytest.raises(AssertionError):
        stats_rule.check(probs, a, b, "offsets")


def test_symmetric_inputs_use_the_spin_averaged_density():
    rng = np.random.default_rng(8)
    probs, a, b = _fake(4, 64, 8, rng, symmetric=True)
    rows = stats_rule.z_table(probs, a, b)
    assert all(len(r) == 2 for r in rows)
    probs, a, b = _fake(4, 64, 8, rng)
    assert all(len(r) == 3 for r in stats_rule.z_table(probs, a, b))


def test_chance_bound_is_the_binomial_tail():
    from scipy.stats import binom
    for n, k in ((256, 3), (104, 2), (1281, 3)):
        bound = stats_rule.allowed_outside(n, k)
        p = 1 - (1 - 0.0027) ** k
        assert binom.sf(bound, n, p) <= 1e-3 < binom.sf(bound - 1, n, p) or bound == int(0.01 * n)
    assert stats_rule.allowed_outside(256, 3) == 8


def test_binned_error_sees_correlation():
    rng = np.random.default_rng(9)
    e = rng.normal(size=4096)
    x = np.empty(4096)
    x[0] = e[0]
    for i in range(1, 4096):  # AR(1), rho = 0.6: the naive error is half the true one
        x[i] = 0.6 * x[i - 1] + e[i]
    naive = x.std(ddof=1) / np.sqrt(len(x))
    assert stats_rule.binned_error(x) > 1.5 * naive
    iid = rng.normal(size=4096)
    assert stats_rule.binned_error(iid) == pytest.approx(iid.std(ddof=1) / 64, rel=0.15)
