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
