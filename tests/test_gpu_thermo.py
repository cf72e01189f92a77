"""Thermodynamics on converged self-consistent solutions (GPU, through the C
ABI): the entropy from dS/dmu = dN/dT over a density scan reproduces the
free-fermion entropy of a trapped lattice site by site, and the interacting
loop converges to the particle-hole symmetric solution at half filling."""
import numpy as np
import pytest

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


def _lattice(n, V0, h=0.0):
    Hu, Hd, coords = wl.trapped_square_onebody(n, n, V0, 0.0, h)
    return Hu - np.diag(np.diag(Hu)), np.stack([np.diag(Hu), np.diag(Hd)]), coords


def _s_of_f(f):
    f = np.clip(f, 1e-300, 1 - 1e-16)
    return -(f * np.log(f) + (1 - f) * np.log1p(-f))


def test_entropy_scan_reproduces_free_fermions(ctx):
    from paper_1006_2716_amd.thermo import entropy_scan
    hop, eps, _ = _lattice(4, 0.3)
    mus = np.linspace(-7.5, 1.0, 86)
    sites = np.arange(16, dtype=np.int32)
    print("entropy scan, 4x4 trap, U = 0, 86 chemical potentials x 2 temperatures, groups of 6", flush=True)
    r = entropy_scan(ctx, hop, 4, eps, eps, 0.0, mus, 38, 42, 0.1, sites, 1, 4, seed=3, n_freq=500, max_iter=2,
                     n_bins=2, mu_group=6)
    E, phi = np.linalg.eigh(hop + np.diag(eps[0]))
    T = r["T"]
    exact = np.stack([2 * (phi ** 2) @ _s_of_f(0.5 * (1 - np.tanh(0.5 * (E - m) / T))) for m in mus])
    err = np.max(np.abs(r["s"] - exact))
    print(f"T = {T:.5f}: max |s - s_exact| = {err:.2e}, total S = {r['s'][-1].sum():.4f}")
    assert err < 3e-3


def test_half_filling_is_particle_hole_symmetric(ctx):
    """Open 4 x 4 lattice, no trap, mu = U/2 (0 after the Hartree shift),
    U = 4, beta = 4: particle-hole symmetry combined with a spin flip
    survives any antiferromagnetic order the loop develops, and in the
    discrete problem n_up + n_dn = 1 holds configuration by configuration, so
    every density is 1 and the real parts of the two spins' self-energies
    (relative to the Hartree shift) cancel, to rounding."""
    from paper_1006_2716_amd.rdmft import RDMFT
    hop, eps, coords = _lattice(4, 0.0)
    r = RDMFT(ctx, hop, 4, eps, 0.0, 4.0, 4.0, 16, n_freq=200)
    try:
        sites = np.arange(16, dtype=np.int32)
        out = r.converge(sites, 200, 8000, seed=21, tol=0.01, max_iter=6, n_bins=16, n_chains=4)
        n = out["density"].sum(axis=1)
        err = np.array([np.hypot(x["n_up_err"], x["n_dn_err"]) for x in out["results"]])
        z = (n - 1.0) / err
        print(f"history {out['history']}, max |z| {np.abs(z).max():.2f}")
        assert np.max(np.abs(n - 1.0)) < 1e-10 and np.abs(z).max() < 1e-6
        sig = r.sigma.cpu().numpy()
        re_sum = np.max(np.abs(sig[0].real + sig[1].real))
        print(f"max |Re(sigma_up + sigma_dn)| {re_sum:.2e}, max |Im sigma| {np.max(np.abs(sig.imag)):.3f}")
        assert re_sum < 1e-10
    finally:
        r.close()


def test_loops_sharing_a_batch_equal_separate_loops(ctx):
    """Two temperatures iterated together (one solver batch per iteration)
    give bitwise the densities and self-energies of separate loops: batch
    composition never changes a result.  The loops' proposal counts cover
    every iteration's solve."""
    from paper_1006_2716_amd.rdmft import RDMFT, converge_together
    hop, eps, _ = _lattice(5, 0.2, h=0.1)
    plain = np.stack([0.5 * (eps[0] + eps[1])] * 2)
    sites = np.arange(25, dtype=np.int32)
    kw = dict(n_bins=4)

    def make():
        return [RDMFT(ctx, hop, 5, eps, 0.3, 4.0, L * 0.25, L, n_freq=100) for L in (14, 18)]

    together = make()
    seen = []  # proposals of every solver call, counted independently of the loops' bookkeeping
    solve = ctx.solve

    def counting(problems):
        res = solve(problems)
        seen.append(sum(int(x["proposals"]) for x in res))
        return res

    ctx.solve = counting
    try:
        outs = converge_together(together, sites, 20, 200, [3, 9], tol=1e-9, max_iter=3, eps_after=plain, **kw)
    finally:
        del ctx.solve
    assert len(seen) == 3 and sum(o["proposals_all"] for o in outs) == sum(seen)
    alone = make()
    try:
        for k, r in enumerate(alone):
            o = r.converge(sites, 20, 200, [3, 9][k], tol=1e-9, max_iter=3, eps_after=plain, **kw)
            assert np.array_equal(o["density"], outs[k]["density"])
            assert np.array_equal(r.sigma.cpu().numpy(), together[k].sigma.cpu().numpy())
            assert o["proposals_all"] == outs[k]["proposals_all"]
            assert o["history_total"] == outs[k]["history_total"] and len(o["history_total"]) == 2
            assert all(t <= 2 * h for t, h in zip(o["history_total"], o["history"]))
    finally:
        for r in together + alone:
            r.close()


def test_find_mu_reaches_the_free_fermion_filling(ctx):
    """U = 0: the bisection lands on the chemical potential whose exact
    free-fermion atom number is the target."""
    from scipy.optimize import brentq
    from paper_1006_2716_amd.thermo import find_mu
    hop, eps, _ = _lattice(6, 0.2)
    sites = np.arange(36, dtype=np.int32)
    E = np.linalg.eigvalsh(hop + np.diag(eps[0]))
    beta, target = 4.0, 20.0

    def atoms(mu):
        return 2 * np.sum(0.5 * (1 - np.tanh(0.5 * beta * (E - mu))))

    exact = brentq(lambda m: atoms(m) - target, -10, 10)
    r = find_mu(ctx, hop, 6, eps, 0.0, 16, beta / 16, sites, target, -6.0, 6.0, 1, 4, seed=1, tol_n=1e-3,
                max_iter=2, n_bins=2)
    print(f"mu {r['mu']:.6f} (exact {exact:.6f}), atoms {r['atoms']:.5f}, {len(r['steps'])} loops")
    assert abs(r["atoms"] - target) < 1e-3
    assert abs(r["mu"] - exact) < 2e-3


def test_grouped_scan_equals_one_mu_at_a_time(ctx):
    """Chemical potentials scanned in groups (their loops and both
    temperatures in one solver batch) give bitwise the densities, errors and
    entropies of the scan one chemical potential at a time, when every loop
    starts from the empty system; with warm starts the grouped scan stays
    within the statistical errors on the free lattice."""
    from paper_1006_2716_amd import hfqmc
    from paper_1006_2716_amd.thermo import density_scan
    hop, eps, _ = _lattice(4, 0.3, h=0.1)
    plain = np.stack([0.5 * (eps[0] + eps[1])] * 2)
    mus = np.linspace(-4.0, 0.0, 7)
    sites = np.arange(16, dtype=np.int32)
    lat = hfqmc.Lattice(ctx, hop, 4)
    try:
        kw = dict(n_freq=100, tol=1e-12, max_iter=2, n_bins=4, warm_start=False)
        one = density_scan(ctx, lat, hop, 4, plain, eps, 4.0, mus, (18, 22), 0.2, sites, 20, 200, 4, **kw)
        print("grouped scan: 7 chemical potentials in groups of 3 (cold starts)", flush=True)
        grp = density_scan(ctx, lat, hop, 4, plain, eps, 4.0, mus, (18, 22), 0.2, sites, 20, 200, 4,
                           mu_group=3, **kw)
    finally:
        lat.close()
    for a in range(2):
        assert np.array_equal(one[0][a], grp[0][a])
        assert np.array_equal(one[1][a], grp[1][a])
        assert one[2][a] == grp[2][a]
        assert np.array_equal(one[4][a], grp[4][a])
        assert np.all(np.isfinite(one[4][a])) and np.all(one[4][a] >= 0)
    assert one[3] == grp[3]
    with pytest.raises(ValueError):
        density_scan(ctx, None, hop, 4, plain, eps, 4.0, mus, (18,), 0.2, sites, 1, 4, 1, mu_group=0)
