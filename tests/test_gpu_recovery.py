"""Numeric failure path and drift control.

A sweep whose Metropolis ratios are not positive numbers is undone and
repeated once from a from-scratch Dyson solve (Eq. (2)) of its starting
fields; a repeat that fails too ends the impurity with HFQMC_ENUMERIC.  The
failure is forced from the host through the library's test hook, which
poisons the diagonal the sweep's ratios read with NaN (no GPU fault is
involved).  A recovered chain takes the decisions of an undisturbed one.

The drift limit halves the interval between from-scratch recomputes while
the measured drift exceeds it and reports HFQMC_ENUMERIC once the interval
is a single sweep.
"""
import json

import numpy as np
import pytest

from paper_1006_2716_amd import workloads as wl

pytestmark = pytest.mark.gpu

ENUMERIC = -5


def _problems(L, delay, n=3, recompute_every=7, n_warmup=6, n_measure=30):
    out = []
    A = wl.chain_adjacency(24)
    for i in range(n):
        Li = L - 3 * i
        beta = min(0.2 * Li, 8.0)
        ws = [wl.weiss_from_onebody(-A - (0.2 * i + 0.1 * s) * np.eye(24), [12], beta, Li)[0] for s in (1, -1)]
        out.append(dict(L=Li, beta=beta, U=5.0 + i, weiss=np.stack(ws), n_warmup=n_warmup, n_measure=n_measure,
                        recompute_every=recompute_every, n_bins=3, seed=71, site=500 + i, delay=delay))
    return out


# (L, delay, forced plan or None): rank-one, delayed fp64, window (forced
# through a tuning-cache entry) and the device-memory kernel
KERNELS = [(64, 1, None), (64, 8, None), (64, 0, (64, 2, 0)), (96, 0, None), (160, 0, None)]


def _ctx(tmp_path, forced, precision=None):
    from paper_1006_2716_amd import hfqmc
    cache = None
    if forced is not None:
        LT, rt, k = forced
        cache = tmp_path / "tune.json"
        cache.write_text(json.dumps({"arch": "gfx950", "entries": [
            {"precision": "fp64", "L_padded": LT, "rt": rt, "k": k, "proposals_per_s": 1.0}]}))
        cache = str(cache)
    kw = {} if precision is None else dict(precision=precision)
    return hfqmc.Context(0, tune_cache=cache, **kw)


@pytest.mark.parametrize("L,delay,forced", KERNELS)
def test_poisoned_sweep_is_recovered(tmp_path, L, delay, forced):
    ctx = _ctx(tmp_path, forced)
    try:
        probs = _problems(L, delay)
        print(f"recovery L={L} delay={delay} forced={forced}", flush=True)
        clean = ctx.solve(probs)
        for r in clean:
            assert r["status"] == 0 and r["recoveries"] == 0
        # one sweep in the warm-up, one that ends with a scheduled recompute
        # (sweep 13 with recompute_every 7), one measured
        for a in (2, 13, 20):
            ctx.debug_poison(a, -1)
            got = ctx.solve(probs)
            for p, g, c in zip(probs, got, clean):
                assert g["status"] == 0, f"sweep {a} L={p['L']}"
                assert g["recoveries"] == 1
                assert np.array_equal(g["fields"], c["fields"])
                assert g["accepts"] == c["accepts"] and g["proposals"] == c["proposals"]
                assert g["nonpositive"] == c["nonpositive"] == 0
                assert np.max(np.abs(g["bins"] - c["bins"])) < 1e-9
        # the repeat poisoned as well: the impurity fails
        ctx.debug_poison(20, 20)
        got = ctx.solve(probs)
        for g in got:
            assert g["status"] == ENUMERIC
            assert g["recoveries"] == 1
        # hook off again: clean results
        ctx.debug_poison(-1, -1)
        again = ctx.solve(probs)
        for g, c in zip(again, clean):
            assert g["status"] == 0 and g["recoveries"] == 0
            assert np.array_equal(g["bins"], c["bins"])
    finally:
        ctx.close()


@pytest.mark.parametrize("L,delay,forced", KERNELS)
def test_drift_limit(tmp_path, L, delay, forced):
    ctx = _ctx(tmp_path, forced)
    try:
        probs = _problems(L, delay, recompute_every=8, n_warmup=4, n_measure=40)
        print(f"drift limit L={L} delay={delay} forced={forced}", flush=True)
        clean = ctx.solve(probs)
        # a limit above the fp64 drift changes nothing
        ctx.set_drift_limit(1e-6)
        got = ctx.solve(probs)
        for g, c in zip(got, clean):
            assert g["status"] == 0
            assert c["max_drift"] < 1e-6
            assert np.array_equal(g["bins"], c["bins"]) and np.array_equal(g["fields"], c["fields"])
        # a limit below any rounding: the interval halves 8 -> 4 -> 2 -> 1,
        # then the next recompute over the limit is an error
        ctx.set_drift_limit(1e-300)
        got = ctx.solve(probs)
        for g, c in zip(got, clean):
            assert g["status"] == ENUMERIC
            assert g["proposals"] == c["proposals"]
        with pytest.raises(Exception):
            ctx.set_drift_limit(-1.0)
        ctx.set_drift_limit(0.0)
        got = ctx.solve(probs)
        for g, c in zip(got, clean):
            assert g["status"] == 0 and np.array_equal(g["bins"], c["bins"])
    finally:
        ctx.close()


def test_drift_limit_schedule_survives_split_launches():
    """A chain served in several launches follows the shortened recompute
    schedule of one launch: same fields and bins as the batch solve."""
    import time
    from paper_1006_2716_amd import hfqmc
    ctx = hfqmc.Context(0)
    try:
        ctx.set_drift_limit(1e-300)  # every recompute halves the interval
        # 30 sweeps, intervals 16, 8, 4, 2: recomputes after sweeps 15, 23, 27, 29
        probs = _problems(64, 1, n=2, recompute_every=16, n_warmup=4, n_measure=26)
        batch = ctx.solve(probs)
        for r in batch:
            assert r["status"] == 0
        ctx.attach_pool(64 << 20)
        ctx.serve_config(quantum_proposals=300)  # a few sweeps per launch
        sites = [ctx.site(p["L"], n_bins=3) for p in probs]
        tickets = {i: ctx.submit(s, p) for i, (s, p) in enumerate(zip(sites, probs))}
        out = {}
        t0 = time.time()
        while len(out) < len(tickets):
            assert time.time() - t0 < 120.0, "serving requests did not finish"
            for k, t in tickets.items():
                if k not in out:
                    r = ctx.poll(t)
                    if r is not None:
                        out[k] = r
            time.sleep(1e-3)
        for k, b in enumerate(batch):
            s = out[k]
            assert s["status"] == 0
            assert np.array_equal(s["fields"], b["fields"])
            assert np.array_equal(s["bins"], b["bins"])
        for s in sites:
            s.close()
    finally:
        ctx.close()
