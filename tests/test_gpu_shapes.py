"""Every compiled kernel shape (tile rows per wave) of the rank-one and the
window-update kernels, and the device-memory kernels, reproduces the
oracle's Markov chain: each is forced through a tuning-cache entry (k = 1:
rank-one, k = 0: window updates, rt = 0: G in device memory) and run on
impurities whose L pads to its class, ragged tails included."""
import json

import numpy as np
import pytest

import oracle
from paper_1006_2716_amd import workloads as wl

pytestmark = pytest.mark.gpu

SHAPES = [(16, 1, 1), (32, 1, 1), (32, 2, 1), (48, 1, 1), (48, 3, 1), (64, 1, 1), (64, 2, 1), (64, 4, 1),
          (80, 1, 1), (96, 1, 1), (96, 2, 1), (96, 3, 1), (112, 1, 1), (128, 1, 1), (128, 2, 1),
          # window updates; the 112-slice class runs on the 128-slice window kernel
          (16, 1, 0), (32, 1, 0), (32, 2, 0), (48, 1, 0), (48, 3, 0), (64, 1, 0), (64, 2, 0), (80, 1, 0),
          (80, 5, 0), (96, 1, 0), (96, 3, 0), (112, 2, 0), (128, 2, 0), (128, 4, 0),
          # G in device memory: window updates (rt 0, k 0) and delayed updates
          (144, 0, 0), (160, 0, 0), (160, 0, 16)]


def _problems(LT):
    out = []
    for i, L in enumerate((LT - 13, LT)):
        A = wl.chain_adjacency(24)
        beta = min(0.2 * L, 8.0)
        ws = [wl.weiss_from_onebody(-A - (0.2 * i + 0.1 * s) * np.eye(24), [12], beta, L)[0] for s in (1, -1)]
        out.append(dict(L=L, beta=beta, U=5.0, weiss=np.stack(ws), n_warmup=4, n_measure=24, recompute_every=7,
                        n_bins=4, seed=61, site=100 * LT + i, delay=0))
    return out


@pytest.mark.parametrize("LT,rt,k", SHAPES)
def test_forced_shape_matches_oracle(tmp_path, LT, rt, k):
    from paper_1006_2716_amd import hfqmc
    print(f"shape LT={LT} rt={rt} k={k}", flush=True)
    cache = tmp_path / "tune.json"
    cache.write_text(json.dumps({"arch": "gfx950", "entries": [
        {"precision": "fp64", "L_padded": LT, "rt": rt, "k": k, "proposals_per_s": 1.0}]}))
    ctx = hfqmc.Context(0, tune_cache=str(cache))
    try:
        assert ctx.plan(LT, 0)[:2] == (rt, k)
        probs = _problems(LT)
        gpu = ctx.solve(probs)
    finally:
        ctx.close()
    ref = oracle.run(probs, n_threads=2)
    for p, g, r in zip(probs, gpu, ref):
        assert np.array_equal(g["fields"], r["fields"]), f"L={p['L']}"
        assert g["accepts"] == r["accepts"]
        assert np.max(np.abs(g["bins"] - r["bins"])) < 1e-9
        assert g["max_drift"] < 1e-8
