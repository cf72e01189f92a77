"""Serving engine on the GPU, through the C ABI: continuous batching of
impurity-solve requests on device-resident sites.

A request is advanced in many short launches (small quanta here, so every
request is split many times), beside whatever else is running.  Its result
must be bitwise the result of hfqmc_solve on the same problem -- alone, in
a mix, and across DMFT iterations that keep fields and G on the device.
"""
import time

import numpy as np
import pytest

import oracle
from paper_1006_2716_amd import serve_load
from paper_1006_2716_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1006_2716_amd import hfqmc
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = hfqmc.Context(0)
    c.attach_pool(256 << 20)
    c.serve_config(quantum_proposals=900)
    yield c
    c.close()


@pytest.fixture(scope="module")
def batch_ctx():
    from paper_1006_2716_amd import hfqmc
    c = hfqmc.Context(0)
    yield c
    c.close()


def _problem(L, mu, it=0, seed=31, site=0, sweeps=60, warm=8, n_bins=4):
    A = wl.chain_adjacency(32)
    H = -A - (mu + 0.02 * it) * np.eye(32)
    g = wl.weiss_from_onebody(H, [16], 0.25 * L, L)[0]
    return dict(L=L, beta=0.25 * L, U=8.0, weiss=np.stack([g, g]), n_warmup=warm, n_measure=sweeps - warm,
                recompute_every=11, n_bins=n_bins, seed=seed, site=site, sweep_offset=it * sweeps, delay=0)


def _wait(ctx, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        assert time.time() - t0 < timeout, "serving requests did not finish"
        for k, t in tickets.items():
            if k not in out:
                r = ctx.poll(t)
                if r is not None:
                    out[k] = r
        time.sleep(1e-3)
    return out


def _same(x, y):
    for k in ("g_up", "g_dn", "bins", "fields"):
        assert np.array_equal(x[k], y[k]), k
    for k in ("proposals", "accepts", "nonpositive", "max_drift", "n_up", "n_dn", "docc", "status"):
        assert x[k] == y[k], k


def test_request_alone_and_in_mix_equal_solve(ctx, batch_ctx):
    Ls = [20, 40, 80, 17, 64, 128, 33, 96, 160, 150]
    probs = [_problem(L, mu=0.1 * i - 0.3, site=i) for i, L in enumerate(Ls)]
    ref = batch_ctx.solve(probs)
    print("alone", flush=True)
    s0 = ctx.site(probs[1]["L"], n_bins=4)
    alone = _wait(ctx, {0: ctx.submit(s0, probs[1])})[0]
    _same(alone, ref[1])
    s0.close()
    print("mix", flush=True)
    sites = [ctx.site(p["L"], n_bins=4) for p in probs]
    tickets = {}
    for i, (s, p) in enumerate(zip(sites, probs)):
        tickets[i] = ctx.submit(s, p)
        time.sleep(0.002 * (i % 3))  # arrivals while others run
    got = _wait(ctx, tickets)
    for i in range(len(probs)):
        _same(got[i], ref[i])
    st = ctx.serve_stats()
    assert st["launches"] > len(probs)  # every request was split over launches
    for s in sites:
        s.close()
    # and the chain is the oracle's
    o = oracle.run([probs[0]])[0]
    assert np.array_equal(got[0]["fields"], o["fields"])
    assert np.max(np.abs(got[0]["bins"] - o["bins"])) < 1e-9


def test_iterations_keep_device_state(ctx, batch_ctx):
    """Iteration j+1 starts from iteration j's final fields with a fresh Dyson
    solve of its new Weiss function."""
    s = ctx.site(40, n_bins=4)
    fields = None
    for it in range(3):
        p = _problem(40, mu=0.2, it=it, site=7)
        r = _wait(ctx, {0: ctx.submit(s, p)})[0]
        q = dict(p)
        if it > 0:
            q["init_fields"] = fields
        _same(r, batch_ctx.solve([q])[0])
        fields = r["fields"]
    s.close()


def test_admission_by_capacity(ctx, batch_ctx):
    """With room for only a few workgroups, requests queue and are admitted as
    others finish; every result is still exact."""
    probs = [_problem(64, mu=-0.2 + 0.05 * i, site=20 + i, sweeps=200) for i in range(12)]
    ref = batch_ctx.solve(probs)
    ctx.serve_config(quantum_proposals=900, capacity_cus=2.0)
    try:
        sites = [ctx.site(64, n_bins=4) for _ in probs]
        tickets = {i: ctx.submit(s, p) for i, (s, p) in enumerate(zip(sites, probs))}
        st = ctx.serve_stats()
        assert st["pending"] > 0 and st["capacity_used"] <= 2.0 + 1e-9
        got = _wait(ctx, tickets)
        for i in range(len(probs)):
            _same(got[i], ref[i])
        for s in sites:
            s.close()
    finally:
        ctx.serve_config(quantum_proposals=900, capacity_cus=0.0)


def test_busy_site_and_cancel(ctx):
    from paper_1006_2716_amd import hfqmc
    s = ctx.site(96, n_bins=4)
    long = _problem(96, mu=0.0, site=3, sweeps=4000, warm=100)
    t = ctx.submit(s, long)
    assert t is not None
    assert ctx.submit(s, _problem(96, mu=0.0, site=3)) is None  # EAGAIN: site busy
    with pytest.raises(hfqmc.HFQMCError):
        s.close()  # EAGAIN while the request runs
    time.sleep(0.01)
    ctx.cancel(t)
    with pytest.raises(hfqmc.HFQMCError):
        ctx.poll(t)  # ENOTFOUND after cancel
    t0 = time.time()
    t2 = None
    while t2 is None:  # the site frees once the running launch retires
        assert time.time() - t0 < 60
        t2 = ctx.submit(s, _problem(96, mu=0.0, site=3, sweeps=20, warm=2))
        time.sleep(1e-3)
    r = _wait(ctx, {0: t2})[0]
    assert r["status"] == 0 and r["proposals"] == 20 * 96
    s.close()


def test_replay_small_stream(ctx, batch_ctx):
    """Timed steps (the default mode): a short Poisson stream over four L
    classes; the last iteration of every site is rechecked against a batch
    solve that starts from the fields the site had before it."""
    sites, arrivals, weiss = wl.serving_requests(n_sites=12, n_iter=3, rate=400.0, Ls=(20, 40, 80, 160),
                                                 weights=(4, 3, 2, 1), sweeps=200, seed=4)
    ctx.serve_config(step_ms=2.0)
    try:
        out = serve_load.replay(ctx, sites, arrivals, weiss, n_iter=3, sweeps=200, warm_first=40, warm_next=10,
                                n_bins=4, timeout_s=120)
    finally:
        ctx.serve_config(quantum_proposals=900)
    assert out["requests"] == 36 and out["p99_ms"] >= out["p50_ms"] > 0
    assert out["proposals"] == sum(200 * s["L"] for s in sites) * 3
    res = out["results"]
    for i, s in enumerate(sites):
        p = serve_load.site_request(s, 2, weiss, 200, 40, 10, n_bins=4)
        p["init_fields"] = res[(i, 1)]["fields"]
        p["delay"] = 0
        _same(res[(i, 2)], batch_ctx.solve([p])[0])
