"""Statistical parity on the GPU: independent Markov chains (different seeds)
on the GPU and in the CPU oracle must agree within their combined Monte Carlo
error, judged over many impurities:

* at least 99 % of the impurities have n_up, n_dn and d within 3 sigma,
* no |z| above 5,
* the mean z^2 over all values lies in [0.7, 1.3]
  (sigma = std(bin means)/sqrt(n_bins) on each side, combined in quadrature).

Also the lattice symmetry of the trap: sites mapped onto each other by the
square's point group have the same Weiss function and, with independent
chains, observables that agree within the same error.
"""
import numpy as np
import pytest

import oracle
from paper_1006_2716_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1006_2716_amd import hfqmc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hfqmc.Context(0)
    yield c
    c.close()


def _z(gpu, ref):
    zs = []
    for g, r in zip(gpu, ref):
        s = oracle.summarize(r["bins"], len(g["g_up"]) - 1)
        row = []
        for key, ekey in (("n_up", "n_up_err"), ("n_dn", "n_dn_err"), ("docc", "docc_err")):
            e = np.hypot(g[ekey], s[ekey])
            row.append((g[key] - s[key]) / e)
        zs.append(row)
    return np.asarray(zs)


def test_independent_chains_agree_within_three_sigma(ctx):
    probs = wl.chain_batch(n_imp=256, Ls=(16, 24, 32), beta=4.0, U_range=(2.0, 6.0), n_warmup=100, n_measure=3200,
                           seed=17)
    for p in probs:
        p["n_bins"] = 32  # 31 degrees of freedom per error: z close to normal
    print(f"{len(probs)} impurities, GPU seed 101, oracle seed 202", flush=True)
    gpu = ctx.solve([dict(p, seed=101) for p in probs])
    ref = oracle.run([dict(p, seed=202) for p in probs], n_threads=16)
    z = _z(gpu, ref)
    ok_rows = np.all(np.abs(z) < 3.0, axis=1)
    print(f"rows within 3 sigma: {ok_rows.mean():.3f}, max |z| {np.abs(z).max():.2f}, mean z^2 {np.mean(z**2):.3f}")
    assert ok_rows.mean() >= 0.99
    assert np.abs(z).max() < 5.0
    assert 0.7 <= np.mean(z ** 2) <= 1.3


def test_trap_symmetry_equivalent_sites(ctx):
    probs, sites, coords = wl.trapped_square(9, 0.2, 4.0, 4.0, 16, 0.0, 0.1, 100, 3200, seed=23)
    for p in probs:
        p["n_bins"] = 16
    where = {tuple(coords[s]): k for k, s in enumerate(sites)}
    pairs = []
    for (x, y), k in where.items():
        for img in ((y, x), (8 - x, y), (x, 8 - y), (8 - y, 8 - x)):
            if img != (x, y) and img in where and (where[img], k) not in pairs:
                pairs.append((k, where[img]))
    assert len(pairs) > 20
    for a, b in pairs:  # the input side of the symmetry
        assert np.max(np.abs(probs[a]["weiss"] - probs[b]["weiss"])) < 1e-12
    res = ctx.solve(probs)
    zs = []
    for a, b in pairs:
        for key, ekey in (("n_up", "n_up_err"), ("n_dn", "n_dn_err"), ("docc", "docc_err")):
            zs.append((res[a][key] - res[b][key]) / np.hypot(res[a][ekey], res[b][ekey]))
    zs = np.asarray(zs)
    print(f"{len(pairs)} symmetric pairs: max |z| {np.abs(zs).max():.2f}, mean z^2 {np.mean(zs**2):.3f}")
    assert np.abs(zs).max() < 5.0
    assert np.mean(np.abs(zs) < 3.0) >= 0.98
