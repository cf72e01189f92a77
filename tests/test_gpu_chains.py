"""Several independent Markov chains per impurity, on the GPU through the C ABI.

Chain j of an impurity keeps its Philox key and sets counter word 3 to j, runs
the full warm-up and its share of the measured sweeps; bin b of the result
pools bin b of every chain.  The oracle's `run_chains` does the same on the
CPU, so the pooled bins agree to rounding and chain 0's final fields agree
exactly.  The serving engine runs each chain as a work item of its own and
must give bitwise the batch result.
"""
import time

import numpy as np
import pytest

import oracle
from oracle import exact as ex
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


@pytest.fixture(scope="module")
def srv():
    from paper_1006_2716_amd import hfqmc
    c = hfqmc.Context(0)
    c.attach_pool(256 << 20)
    c.serve_config(quantum_proposals=700)
    yield c
    c.close()


def _problem(L, U, mu, n_chains, seed=3, site=0, n_warmup=6, n_measure=41, n_bins=4):
    A = wl.chain_adjacency(24)
    ws = []
    for h in (0.15, -0.15):
        ws.append(wl.weiss_from_onebody(-A - (mu + h) * np.eye(24), [12], min(0.2 * L, 10.0), L)[0])
    return dict(L=L, beta=min(0.2 * L, 10.0), U=U, weiss=np.stack(ws), n_warmup=n_warmup, n_measure=n_measure,
                recompute_every=9, n_bins=n_bins, seed=seed, site=site, n_chains=n_chains)


def _check_pooled(g, p, tol=1e-9):
    pooled, counts, parts = oracle.run_chains(p, max(1, p.get("n_chains", 1)), n_threads=8)
    assert g["status"] == 0
    assert np.array_equal(g["fields"], parts[0]["fields"]), f"L={p['L']}: chain 0 trajectory differs"
    assert g["proposals"] == sum(r["proposals"] for r in parts)
    assert g["accepts"] == sum(r["accepts"] for r in parts)
    assert np.max(np.abs(g["bins"] - pooled)) < tol, f"L={p['L']}"
    s = oracle.summarize(pooled, p["L"])
    for k in ("n_up", "n_dn", "docc", "n_up_err", "docc_err"):
        assert abs(g[k] - s[k]) < tol, k


# ---------------------------------------------------------------- batch path
def test_pooled_chains_match_oracle(ctx):
    """Register-tile (small, bin-accumulating and plain) and device-memory
    kernels, chain counts that do and do not divide n_measure."""
    cases = [(20, 3), (40, 4), (64, 2), (100, 3), (150, 2)]
    probs = [_problem(L, U=4.0 + i, mu=0.1 * i - 0.2, n_chains=nc, site=i) for i, (L, nc) in enumerate(cases)]
    print("pooled chains", [(p["L"], p["n_chains"]) for p in probs], flush=True)
    gpu = ctx.solve(probs)
    for g, p in zip(gpu, probs):
        _check_pooled(g, p)


def test_largest_chain_count(ctx):
    """64 chains (the most a problem may have; 191 measured sweeps: 63 chains
    run 3, the last 2), on a register and a device-memory kernel."""
    probs = [_problem(L, U=5.0, mu=0.05, n_chains=64, site=30 + L, n_warmup=3, n_measure=64 * 2 + 63, n_bins=2)
             for L in (16, 144)]
    print("64 chains", [p["L"] for p in probs], flush=True)
    gpu = ctx.solve(probs)
    for g, p in zip(gpu, probs):
        _check_pooled(g, p)


def test_one_chain_is_the_plain_run(ctx):
    p = _problem(48, U=6.0, mu=0.1, n_chains=0)
    a = ctx.solve([p])[0]
    b = ctx.solve([dict(p, n_chains=1)])[0]
    assert np.array_equal(a["bins"], b["bins"]) and np.array_equal(a["fields"], b["fields"])
    r = oracle.run([p])[0]
    assert np.array_equal(a["fields"], r["fields"])
    assert np.max(np.abs(a["bins"] - r["bins"])) < 1e-9


def test_chains_beside_single_chain_problems(ctx):
    """A multi-chain problem in a batch with other problems gives bitwise its
    result alone (chains are ordinary work items of their kernel class)."""
    multi = _problem(64, U=5.0, mu=0.0, n_chains=5, site=7, n_measure=60)
    others = [_problem(L, U=6.0, mu=0.3, n_chains=0, site=20 + L) for L in (16, 64, 96)]
    alone = ctx.solve([multi])[0]
    mixed = ctx.solve(others[:2] + [multi] + others[2:])[2]
    assert np.array_equal(alone["bins"], mixed["bins"])
    assert np.array_equal(alone["fields"], mixed["fields"])


def test_pooled_chains_match_enumeration(ctx):
    """Statistics: 16 chains of one two-site impurity against the exact
    enumeration of every field configuration."""
    L, beta, U, mu, V, eb = 8, 2.0, 4.0, 1.0, 0.8, 0.4
    p = wl.two_site_problem(L, beta, U, mu, V, eb, h=0.2, n_warmup=300, n_measure=64000, seed=77, n_bins=32)
    p["n_chains"] = 16
    lam = oracle.lam(beta / L, U)
    vals, _, _ = ex.enumerate_fields(p["weiss"][0], p["weiss"][1], lam)
    g = ctx.solve([p])[0]
    zs = [(g["n_up"] - vals[2 * L + 2]) / g["n_up_err"], (g["n_dn"] - vals[2 * L + 3]) / g["n_dn_err"],
          (g["docc"] - vals[2 * L + 4]) / g["docc_err"]]
    print("z", zs)
    assert max(abs(z) for z in zs) < 4.0, zs


def test_invalid_chain_counts_raise(ctx):
    from paper_1006_2716_amd import hfqmc
    p = _problem(16, U=4.0, mu=0.0, n_chains=4)
    with pytest.raises(hfqmc.HFQMCError):
        ctx.solve([dict(p, n_chains=65)])
    with pytest.raises(hfqmc.HFQMCError):
        ctx.solve([dict(p, n_chains=-1)])
    with pytest.raises(hfqmc.HFQMCError):  # 11 chains x 4 bins > 41 measured sweeps
        ctx.solve([dict(p, n_chains=11)])


# ---------------------------------------------------------------- serving
def _wait(c, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        assert time.time() - t0 < timeout, "serving requests did not finish"
        for k, t in tickets.items():
            if k not in out:
                r = c.poll(t)
                if r is not None:
                    out[k] = r
        time.sleep(1e-3)
    return out


def _same(x, y):
    for k in ("g_up", "g_dn", "bins", "fields"):
        assert np.array_equal(x[k], y[k]), k
    for k in ("proposals", "accepts", "nonpositive", "max_drift", "n_up", "n_dn", "docc", "status"):
        assert x[k] == y[k], k


def test_serving_chains_equal_batch(srv, ctx):
    cases = [(32, 3), (64, 4), (96, 1), (160, 3)]
    probs = [_problem(L, U=6.0, mu=0.1 * i, n_chains=nc, site=i, n_measure=50) for i, (L, nc) in enumerate(cases)]
    ref = ctx.solve(probs)
    print("serving chains", cases, flush=True)
    sites = [srv.site(p["L"], n_bins=p["n_bins"], n_chains=p["n_chains"]) for p in probs]
    try:
        got = _wait(srv, {i: srv.submit(s, p) for i, (s, p) in enumerate(zip(sites, probs))})
        for i in range(len(probs)):
            _same(got[i], ref[i])
        # next iteration from given fields: every chain starts from them
        init = np.where(np.arange(64) % 2 == 0, 1, -1).astype(np.int8)
        p2 = dict(probs[1], init_fields=init, sweep_offset=50)
        _same(_wait(srv, {0: srv.submit(sites[1], p2)})[0], ctx.solve([p2])[0])
    finally:
        for s in sites:
            s.close()


def test_serving_site_chain_count_must_match(srv):
    from paper_1006_2716_amd import hfqmc
    p = _problem(32, U=4.0, mu=0.0, n_chains=2)
    s = srv.site(32, n_bins=4, n_chains=3)
    try:
        with pytest.raises(hfqmc.HFQMCError):
            srv.submit(s, p)
    finally:
        s.close()
