"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, and its pure-host calls behave."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1006_2716_amd import hfqmc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hfqmc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hfqmc_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("hfqmc_lambda", "hfqmc_create", "hfqmc_solve", "hfqmc_workspace_size", "hfqmc_site_force_flips"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(hfqmc.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("dtau,U", [(0.25, 4.0), (0.125, 12.0), (0.2, 8.0), (1.0, 1e-9)])
def test_lambda_defining_identity(dtau, U):
    lam = hfqmc.lam(dtau, U)
    assert np.cosh(lam) == pytest.approx(np.exp(0.5 * dtau * U), rel=1e-14)


def test_lambda_rejects_bad_input():
    with pytest.raises(hfqmc.HFQMCError) as e:
        hfqmc.lam(0.0, 4.0)
    assert e.value.status == hfqmc.EINVAL
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.lam(0.25, -1.0)


def test_site_bytes_grows_with_L():
    b16 = hfqmc.site_bytes(16)
    b64 = hfqmc.site_bytes(64)
    b128 = hfqmc.site_bytes(128)
    b160 = hfqmc.site_bytes(160)
    assert b16 < b64 < b128 < b160
    # G of both spins plus its drift snapshot dominate: 4 x L x L doubles
    assert b128 >= 4 * 128 * 128 * 8 and b160 >= 4 * 160 * 160 * 8
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.site_bytes(161)
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.site_bytes(0)


def test_site_bytes_per_chain():
    one = hfqmc.site_bytes(96, 16)
    assert hfqmc.site_bytes(96, 16, 0) == one  # 0 and 1 both mean one chain
    four = hfqmc.site_bytes(96, 16, 4)
    # every chain holds its own G, fields, bins and status; Weiss and buffers are shared
    per_chain = four - one
    assert per_chain % 3 == 0 and per_chain // 3 >= 4 * 96 * 96 * 8
    assert four < 4 * one
    for bad in (-1, 65):
        with pytest.raises(hfqmc.HFQMCError):
            hfqmc.site_bytes(96, 16, bad)


def test_null_context_is_rejected():
    lib = hfqmc.lib()
    assert lib.hfqmc_workspace_size(None, None, 0, None) == hfqmc.EINVAL
    assert lib.hfqmc_run(None) == hfqmc.EINVAL
    assert lib.hfqmc_collect(None, None) == hfqmc.EINVAL


def test_extrapolation_fit_matches_the_oracle():
    """Host-only library arithmetic: the dtau -> 0 fit against the oracle's
    least squares, weighted and unweighted, orders 0 .. 2."""
    from oracle import trotter as tr
    rng = np.random.default_rng(4)
    d = np.array([0.25, 0.2, 0.1667, 0.125, 0.1])
    y = 0.12 + 0.3 * d ** 2 - 0.5 * d ** 4 + rng.normal(scale=1e-3, size=d.size)
    e = rng.uniform(5e-4, 2e-3, size=d.size)
    for order in (0, 1, 2):
        c, ce = hfqmc.extrapolate(d, y, e, order)
        rc, rce = tr.fit(d, y, e, order)
        assert np.allclose(c, rc, rtol=1e-10, atol=1e-13) and np.allclose(ce, rce, rtol=1e-10)
        c, ce = hfqmc.extrapolate(d, y, None, order)
        assert ce is None and np.allclose(c, tr.fit(d, y, None, order)[0], rtol=1e-10, atol=1e-13)


def test_extrapolation_rejects_bad_input():
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.extrapolate([0.1, 0.1], [1.0, 1.1], None, 1)  # one distinct dtau
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.extrapolate([0.1, 0.2], [1.0, 1.1], None, 2)  # too few points
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.extrapolate([0.1, -0.2], [1.0, 1.1], None, 1)
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.extrapolate([0.1, 0.2], [1.0, 1.1], [0.1, 0.0], 1)


def test_entropy_integral_matches_the_oracle():
    from oracle import thermo as th
    rng = np.random.default_rng(8)
    mu = np.sort(rng.uniform(-5, 2, size=40))
    a = rng.uniform(0, 2, size=(40, 7))
    b = a + rng.normal(scale=0.01, size=a.shape)
    s = hfqmc.entropy(mu, a, b, 0.2, 0.22)
    assert np.allclose(s, th.entropy_from_densities(mu, a, b, 0.2, 0.22), rtol=1e-12, atol=1e-14)
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.entropy(mu[::-1], a, b, 0.2, 0.22)
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.entropy(mu, a, b, 0.22, 0.2)


def test_lattice_bytes_host_rules():
    lib = hfqmc.lib()
    b = C.c_size_t()
    assert lib.hfqmc_lattice_bytes(441, 21, C.byref(b)) == hfqmc.OK
    # 21 blocks of 21 x 21 doubles, 20 couplings of 21, then 441 int32 site slots (256-byte aligned parts)
    hop = 8 * (21 * 21 * 21 + 20 * 21)
    assert b.value == (hop + 255) // 256 * 256 + (4 * 441 + 255) // 256 * 256
    for n, layer in ((441, 65), (440, 21), (0, 1), (20, 0)):
        assert lib.hfqmc_lattice_bytes(n, layer, C.byref(b)) == hfqmc.EINVAL


def test_problem_marshalling_places_every_field():
    """The packed Problem structs hold each problem's scalars, and their
    pointers reach that problem's Weiss samples and initial fields (read back
    through ctypes, as the library reads them)."""
    rng = np.random.default_rng(4)
    probs = []
    for i, L in enumerate((5, 16, 1, 33, 7)):
        p = dict(L=L, beta=1.0 + i, U=0.5 * i, weiss=rng.random((2, L)), n_warmup=10 + i, n_measure=100 + i,
                 n_bins=2 + i, seed=2 ** 63 + i if i == 3 else i, site=7 * i)
        if i in (1, 3):
            p["init_fields"] = rng.choice([-1, 1], size=L)
        if i == 2:
            p.update(recompute_every=3, sweep_offset=-5, delay=4, n_chains=2, seed=-1)
        probs.append(p)
    P = hfqmc._Problems(probs)
    assert P.n == 5
    for i, p in enumerate(probs):
        s = P.arr[i]
        L = p["L"]
        assert (s.L, s.beta, s.U, s.n_warmup, s.n_measure, s.n_bins) == (L, p["beta"], p["U"], p["n_warmup"],
                                                                        p["n_measure"], p["n_bins"])
        assert s.seed == p["seed"] % 2 ** 64 and s.site_id == p["site"]
        assert (s.recompute_every, s.sweep_offset, s.delay, s.n_chains) == (
            p.get("recompute_every", 50), p.get("sweep_offset", 0), p.get("delay", 0), p.get("n_chains", 0))
        for sp in range(2):
            assert [s.weiss[sp][k] for k in range(L)] == p["weiss"][sp].tolist()
        if "init_fields" in p:
            assert [s.init_fields[k] for k in range(L)] == p["init_fields"].tolist()
        else:
            assert not s.init_fields
    with pytest.raises(ValueError):
        hfqmc._Problems([dict(probs[0], weiss=np.zeros((2, 4)))])
    with pytest.raises(ValueError):
        hfqmc._Problems([dict(probs[0], init_fields=np.ones(4))])
    assert hfqmc._Problems([]).n == 0


def test_result_buffers_are_disjoint_and_read_back():
    """Each Result struct points at its own output arrays; values written
    through those pointers come back in to_list()."""
    probs = [dict(L=L, n_bins=nb) for L, nb in ((3, 2), (16, 4), (1, 3))]
    R = hfqmc._Results(probs)
    for i, p in enumerate(probs):
        r = R.arr[i]
        L, nb = p["L"], p["n_bins"]
        for sp in range(2):
            for k in range(L + 1):
                r.g[sp][k] = 1000 * i + 100 * sp + k
                r.g_err[sp][k] = -(1000 * i + 100 * sp + k)
        for k in range(nb * (2 * (L + 1) + 3)):
            r.bins[k] = 10000 * i + k
        for k in range(L):
            r.final_fields[k] = 1 if (i + k) % 2 else -1
        r.n[0], r.n[1], r.proposals, r.status = 0.25 + i, 0.5 + i, 17 * i, -i
    out = R.to_list()
    for i, (p, o) in enumerate(zip(probs, out)):
        L, nb = p["L"], p["n_bins"]
        assert o["g_up"].tolist() == [1000 * i + k for k in range(L + 1)]
        assert o["g_dn"].tolist() == [1000 * i + 100 + k for k in range(L + 1)]
        assert o["g_dn_err"].tolist() == [-(1000 * i + 100 + k) for k in range(L + 1)]
        assert o["bins"].shape == (nb, 2 * (L + 1) + 3)
        assert o["bins"].reshape(-1).tolist() == [10000 * i + k for k in range(o["bins"].size)]
        assert o["fields"].tolist() == [1 if (i + k) % 2 else -1 for k in range(L)]
        assert (o["n_up"], o["n_dn"], o["proposals"], o["status"]) == (0.25 + i, 0.5 + i, 17 * i, -i)
        assert isinstance(o["proposals"], int) and isinstance(o["n_up"], float)
    assert hfqmc._Results([]).to_list() == []


def test_scan_solver_seeds_never_repeat():
    """Every (chemical potential, temperature, iteration) loop of an entropy
    scan, and every bisection step of the chemical-potential search, draws a
    solver seed of its own: the Philox key is (seed, site), so a repeated
    seed would replay another loop's fields and uniforms."""
    from paper_1006_2716_amd import thermo
    max_iter, n_mu = thermo.SEED_STRIDE, 60
    seeds = [thermo.loop_seed(5, k, a) + it for k in range(n_mu) for a in range(thermo.MAX_TEMPERATURES)
             for it in range(max_iter)]
    assert len(set(seeds)) == len(seeds)
    steps = [5 + thermo.SEED_STRIDE * s + it for s in range(40) for it in range(max_iter)]
    assert len(set(steps)) == len(steps)
    with pytest.raises(ValueError):
        thermo._check_seed_room(thermo.SEED_STRIDE + 1)
    with pytest.raises(ValueError):
        thermo._check_seed_room(5, thermo.MAX_TEMPERATURES + 1)
