"""Delayed rank-k updates (G = G0 + A B^T flushed on the matrix cores).

fp64 flushes reproduce the oracle's Sherman-Morrison chain up to rounding:
same Philox stream, same decisions, so the field trajectories coincide and
the observables agree element by element.  Mixed precision (fp32 products
added into fp64 G) has no exact reference; its statistical comparison with
the fp64 oracle is in test_gpu_zstatistics_configs.py.
"""
import numpy as np
import pytest

import oracle
from paper_1006_2716_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _chain(L, U, mu, beta, seed, site, n_warmup, n_measure, n_bins=4, delay=1, h=0.0):
    A = wl.chain_adjacency(24)
    ws = []
    for sigma in (+1, -1):
        H = -A - (mu + sigma * h) * np.eye(24)
        ws.append(wl.weiss_from_onebody(H, [12], beta, L)[0])
    return dict(L=L, beta=beta, U=U, weiss=np.stack(ws), n_warmup=n_warmup, n_measure=n_measure,
                recompute_every=50, n_bins=n_bins, seed=seed, site=site, delay=delay)


@pytest.fixture(scope="module")
def ctx64():
    from paper_1006_2716_amd import hfqmc
    c = hfqmc.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("delay", [2, 4, 8, 16, 32])
def test_delayed_fp64_matches_oracle_trajectory(ctx64, delay):
    print(f"delayed fp64 k={delay}", flush=True)
    Ls = [17, 32, 40, 48, 64, 80, 96, 128]
    probs = [_chain(L, U=5.0 + 0.5 * i, mu=0.2 * i - 0.6, beta=min(0.2 * L, 10.0), seed=13, site=i,
                    n_warmup=4, n_measure=40, delay=delay) for i, L in enumerate(Ls)]
    probs[0]["recompute_every"] = 7
    gpu = ctx64.solve(probs)
    ref = oracle.run(probs, n_threads=8)
    for p, g, r in zip(probs, gpu, ref):
        assert g["status"] == 0
        assert np.array_equal(g["fields"], r["fields"]), f"L={p['L']}"
        assert g["accepts"] == r["accepts"] and g["proposals"] == r["proposals"]
        assert np.max(np.abs(g["bins"] - r["bins"])) < 1e-9, f"L={p['L']}"
        assert g["max_drift"] < 1e-8


def test_delayed_fp64_full_headline_sample(ctx64):
    """The L = 64 batch with k = 16, three impurities recomputed by the oracle."""
    probs = wl.chain_batch_L64(n_imp=64)
    for p in probs:
        p["delay"] = 16
    gpu = ctx64.solve(probs)
    idx = [0, 31, 63]
    ref = oracle.run([probs[i] for i in idx], n_threads=3)
    for i, r in zip(idx, ref):
        assert np.array_equal(gpu[i]["fields"], r["fields"])
        assert np.max(np.abs(gpu[i]["bins"] - r["bins"])) < 1e-9
