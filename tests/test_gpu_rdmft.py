"""Real-space DMFT self-consistency on the GPU, through the C ABI, against the
dense oracle (``oracle/rdmft.py``): lattice Green function (Eq. (2)), Weiss
functions and their tau samples, self-energy update, and whole iterations
whose impurity solves draw the same Philox streams on both sides."""
import numpy as np
import pytest

import oracle
from oracle import rdmft as rd
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


def _lattice(nx, ny, V0=0.05, mu_eff=0.0, h=0.1):
    """Open nx x ny trap, sites numbered x * ny + y: layers are rows of ny sites."""
    Hu, Hd, coords = wl.trapped_square_onebody(nx, ny, V0, mu_eff, h)
    hop = Hu - np.diag(np.diag(Hu))
    eps = np.stack([np.diag(Hu), np.diag(Hd)]) + mu_eff
    return hop, eps, mu_eff, (Hu, Hd)


def _sigma(rng, nf, N, beta):
    """A causal-looking self-energy: Im sigma <= 0 at positive frequencies."""
    w = rd.matsubara(beta, nf)
    a = rng.uniform(0.5, 3.0, size=(2, 1, N))
    return rng.normal(scale=0.5, size=(2, 1, N)) + a / (1j * w[None, :, None] + rng.uniform(-1, 1, size=(2, 1, N)))


def _t(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda:0", dtype=dtype)


@pytest.mark.parametrize("nx,ny", [(5, 7), (3, 20), (4, 41), (2, 64), (1, 37), (6, 1)])
def test_lattice_green_matches_dense_inverse(ctx, nx, ny):
    """Every padded layer width (16/32/48/64), one layer (a dense inverse),
    layers of one site (a chain)."""
    from paper_1006_2716_amd import hfqmc
    import torch
    print(f"lattice green {nx}x{ny}", flush=True)
    hop, eps, mu, _ = _lattice(nx, ny, V0=0.2, mu_eff=0.3)
    N, beta, nf = nx * ny, 5.0, 6
    sig = _sigma(np.random.default_rng(nx * 100 + ny), nf, N, beta)
    lat = hfqmc.Lattice(ctx, hop, ny)
    try:
        g = lat.green(nf, beta, mu, _t(eps), _t(sig, torch.complex128)).cpu().numpy()
    finally:
        lat.close()
    ref = rd.lattice_local_green(hop, eps, mu, sig, beta)
    assert np.max(np.abs(g - ref) / np.abs(ref)) < 1e-11


@pytest.mark.parametrize("n", [21, 41])
def test_lattice_green_full_size_sampled(ctx, n):
    """The 21 x 21 and 41 x 41 traps at 500 frequencies; the oracle inverts
    four sampled frequencies of each spin."""
    from paper_1006_2716_amd import hfqmc
    import torch
    print(f"lattice green {n}x{n}, 500 frequencies", flush=True)
    hop, eps, mu, _ = _lattice(n, n, V0=0.05 if n == 21 else 0.02, mu_eff=0.0 if n == 21 else 3.154)
    N, beta, nf = n * n, 10.0, 500
    sig = _sigma(np.random.default_rng(n), nf, N, beta)
    lat = hfqmc.Lattice(ctx, hop, n)
    try:
        g = lat.green(nf, beta, mu, _t(eps), _t(sig, torch.complex128)).cpu().numpy()
    finally:
        lat.close()
    idx = [0, 1, 250, 499]
    ref = rd.lattice_local_green(hop, eps, mu, sig[:, idx], beta, n_index=idx)
    assert np.max(np.abs(g[:, idx] - ref) / np.abs(ref)) < 1e-11


def test_weiss_matches_oracle_and_the_trap_workload(ctx):
    """sigma = 0 on the 21 x 21 trap: the Weiss functions' tau samples equal
    the oracle's transform, and the eigen-decomposition Weiss functions the
    trapped-cloud workload is built from (within the Matsubara truncation)."""
    from paper_1006_2716_amd import hfqmc
    import torch
    probs, sites, coords = wl.trapped_square(21, 0.05, 8.0, 10.0, 40, 0.0, 0.1, 10, 100, seed=2)
    hop, eps, mu, _ = _lattice(21, 21, V0=0.05, mu_eff=0.0, h=0.1)
    N, beta, nf, L = 441, 10.0, 500, 40
    lat = hfqmc.Lattice(ctx, hop, 21)
    try:
        sig0 = torch.zeros((2, nf, N), dtype=torch.complex128, device="cuda:0")
        e_t = _t(eps)
        gl = lat.green(nf, beta, mu, e_t, sig0)
        w_iw, w_tau = lat.weiss(nf, beta, mu, L, e_t, gl, sig0, sites)
        w_iw, w_tau, gl = w_iw.cpu().numpy(), w_tau.cpu().numpy(), gl.cpu().numpy()
    finally:
        lat.close()
    assert w_tau.shape == (len(sites), 2, L)
    # the oracle's transforms of the GPU's local Green function, sampled sites
    taus = np.arange(L) * (beta / L)
    for j in (0, len(sites) // 2, len(sites) - 1):
        i = sites[j]
        for s in range(2):
            W = rd.weiss_iw(gl[s, :, i], np.zeros(nf))
            assert np.max(np.abs(w_iw[s, :, j] - W)) < 1e-13
            ref = rd.tau_from_iw(W, eps[s, i] - mu, beta, taus)
            assert np.max(np.abs(w_tau[j, s] - ref)) < 1e-12
    # against the workload's exact U = 0 Weiss functions (eigen-decomposition)
    exact = np.stack([p["weiss"] for p in probs])
    assert np.max(np.abs(w_tau - exact)) < 2e-5


def test_sigma_update_matches_oracle(ctx):
    """Self-energy of sampled sites from real solver output (a short solve of
    the trapped cloud's Weiss functions)."""
    from paper_1006_2716_amd import hfqmc
    import torch
    nx, L, beta, U, nf = 7, 24, 6.0, 6.0, 300
    hop, eps, mu, _ = _lattice(nx, nx, V0=0.1, mu_eff=0.2, h=0.1)
    N = nx * nx
    sites = np.arange(0, N, 3, dtype=np.int32)
    rng = np.random.default_rng(5)
    sig = 0.3 * _sigma(rng, nf, N, beta)
    lat = hfqmc.Lattice(ctx, hop, nx)
    try:
        s_t = _t(sig, torch.complex128)
        e_t = _t(eps)
        gl = lat.green(nf, beta, mu, e_t, s_t)
        w_iw, w_tau = lat.weiss(nf, beta, mu, L, e_t, gl, s_t, sites)
        w_tau_h = w_tau.cpu().numpy()
        probs = [dict(L=L, beta=beta, U=U, weiss=w_tau_h[j], n_warmup=20, n_measure=200, recompute_every=20,
                      n_bins=4, seed=9, site=int(sites[j])) for j in range(len(sites))]
        res = ctx.solve(probs)
        gimp = np.stack([np.stack([r["g_up"], r["g_dn"]]) for r in res])
        dens = np.array([[r["n_up"], r["n_dn"]] for r in res])
        for mix in (1.0, 0.5):
            out = s_t.clone()
            lat.sigma_update(nf, beta, mu, U, L, e_t, sites, w_iw, _t(gimp), _t(dens), mix, out)
            out = out.cpu().numpy()
            w_iw_h = w_iw.cpu().numpy()
            untouched = np.setdiff1d(np.arange(N), sites)
            assert np.array_equal(out[:, :, untouched], sig[:, :, untouched])
            for j in range(len(sites)):
                i = sites[j]
                for s in range(2):
                    new = rd.sigma_update(w_iw_h[s, :, j], eps[s, i] - mu, gimp[j, s], dens[j, 1 - s], U, beta)
                    ref = mix * new + (1 - mix) * sig[s, :, i]
                    assert np.max(np.abs(out[s, :, i] - ref)) < 1e-9 * max(1.0, np.max(np.abs(ref))), (j, s)
    finally:
        lat.close()


def _oracle_iteration(hop, eps, mu, U, beta, L, nf, sigma, sites, n_warmup, n_measure, seed, n_bins):
    gl = rd.lattice_local_green(hop, eps, mu, sigma, beta)
    taus = np.arange(L) * (beta / L)
    weiss_iw, weiss_tau = [], []
    for i in sites:
        wi = [rd.weiss_iw(gl[s, :, i], sigma[s, :, i]) for s in range(2)]
        weiss_iw.append(wi)
        weiss_tau.append(np.stack([rd.tau_from_iw(wi[s], eps[s, i] - mu, beta, taus) for s in range(2)]))
    probs = [dict(L=L, beta=beta, U=U, weiss=weiss_tau[j], n_warmup=n_warmup, n_measure=n_measure,
                  recompute_every=50, n_bins=n_bins, seed=seed, site=int(sites[j])) for j in range(len(sites))]
    res = oracle.run(probs, n_threads=8)
    new = sigma.copy()
    for j, i in enumerate(sites):
        s_ = oracle.summarize(res[j]["bins"], L)
        gi = [s_["g_up"], s_["g_dn"]]
        dn = [s_["n_up"], s_["n_dn"]]
        for s in range(2):
            new[s, :, i] = rd.sigma_update(weiss_iw[j][s], eps[s, i] - mu, gi[s], dn[1 - s], U, beta)
    return new, np.stack(weiss_tau), res


def test_two_iterations_match_oracle(ctx):
    """Open 4 x 4 lattice, U = 4, beta = 4, L = 16: two full iterations, GPU
    path against the oracle's composition; identical Philox streams give
    identical field trajectories, so self-energies agree to rounding."""
    from paper_1006_2716_amd.rdmft import RDMFT
    hop, eps, mu, _ = _lattice(4, 4, V0=0.0, mu_eff=0.0, h=0.1)
    U, beta, L, nf = 4.0, 4.0, 16, 100
    sites = np.arange(16, dtype=np.int32)
    r = RDMFT(ctx, hop, 4, eps, mu, U, beta, L, n_freq=nf)
    try:
        sig_o = np.zeros((2, nf, 16), dtype=np.complex128)
        for it in range(2):
            print(f"iteration {it}", flush=True)
            g = r.iterate(sites, n_warmup=20, n_measure=400, seed=11 + it, n_bins=8)
            sig_o, wt_o, res_o = _oracle_iteration(hop, eps, mu, U, beta, L, nf, sig_o, sites, 20, 400, 11 + it, 8)
            assert np.max(np.abs(g["weiss_tau"] - wt_o)) < 1e-12
            for a, b in zip(g["results"], res_o):
                assert np.array_equal(a["fields"], b["fields"])
            sig_g = r.sigma.cpu().numpy()
            assert np.max(np.abs(sig_g - sig_o)) < 1e-8
    finally:
        r.close()


def test_U0_is_a_fixed_point(ctx):
    """U = 0: the solver returns the Weiss function, the self-energy stays zero
    and the densities are the non-interacting lattice's."""
    from paper_1006_2716_amd.rdmft import RDMFT
    hop, eps, mu, (Hu, Hd) = _lattice(5, 6, V0=0.1, mu_eff=0.3, h=0.1)
    r = RDMFT(ctx, hop, 6, eps, mu, 0.0, 4.0, 20, n_freq=400)
    try:
        sites = np.arange(30, dtype=np.int32)
        g = r.iterate(sites, n_warmup=2, n_measure=8, seed=3, n_bins=2)
        assert np.max(np.abs(r.sigma.cpu().numpy())) < 1e-10
        n0 = np.stack([wl.densities_from_onebody(Hu, 4.0), wl.densities_from_onebody(Hd, 4.0)], axis=1)
        assert np.max(np.abs(g["density"] - n0)) < 2e-5  # Matsubara truncation of the Weiss samples
    finally:
        r.close()


def test_invalid_lattices_and_lists_raise(ctx):
    from paper_1006_2716_amd import hfqmc
    import torch
    hop, eps, mu, _ = _lattice(4, 5)
    ring = hop.copy()
    ring[0, 19] = ring[19, 0] = -1.0  # periodic wrap: not layered
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.Lattice(ctx, ring, 5)
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.Lattice(ctx, hop, 3)  # 3 does not divide 20
    diag = hop.copy()
    diag[0, 6] = diag[6, 0] = -0.5  # next-nearest neighbour across layers
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.Lattice(ctx, diag, 5)
    big = np.zeros((130, 130))
    with pytest.raises(hfqmc.HFQMCError):
        hfqmc.Lattice(ctx, big, 65)
    lat = hfqmc.Lattice(ctx, hop, 5)
    other = hfqmc.Context(0)
    try:
        s0 = torch.zeros((2, 4, 20), dtype=torch.complex128, device="cuda:0")
        ws = torch.empty(lat.workspace_size(4), dtype=torch.uint8, device="cuda:0")
        gl = torch.empty((2, 4, 20), dtype=torch.complex128, device="cuda:0")
        e_t = _t(eps)
        st = hfqmc.lib().hfqmc_lattice_green(other.h, lat.h, 4, 3.0, mu, hfqmc._VP(e_t.data_ptr()),
                                             hfqmc._VP(s0.data_ptr()), hfqmc._VP(gl.data_ptr()),
                                             hfqmc._VP(ws.data_ptr()), ws.numel())
        assert st == hfqmc.EINVAL  # a lattice works only with the context that created it
        gl = lat.green(4, 3.0, mu, _t(eps), s0)
        with pytest.raises(hfqmc.HFQMCError):
            lat.weiss(4, 3.0, mu, 8, _t(eps), gl, s0, [0, 20])
        w_iw, _ = lat.weiss(4, 3.0, mu, 8, _t(eps), gl, s0, [0, 1])
        with pytest.raises(hfqmc.HFQMCError):
            lat.sigma_update(4, 3.0, mu, 1.0, 8, _t(eps), [1, 1], w_iw, torch.zeros((2, 2, 9), dtype=torch.float64,
                             device="cuda:0"), torch.zeros((2, 2), dtype=torch.float64, device="cuda:0"), 1.0, s0)
    finally:
        lat.close()
        other.close()


def test_iterations_from_previous_fields_match_oracle(ctx):
    """keep_fields: the second iteration starts every site from its first
    iteration's final fields (short warm-up); the oracle run from the same
    fields gives the same chains."""
    from paper_1006_2716_amd.rdmft import RDMFT
    hop, eps, mu, _ = _lattice(3, 4, V0=0.1, mu_eff=0.2, h=0.1)
    U, beta, L, nf = 5.0, 4.0, 16, 100
    sites = np.arange(12, dtype=np.int32)
    r = RDMFT(ctx, hop, 4, eps, mu, U, beta, L, n_freq=nf)
    try:
        first = r.iterate(sites, 30, 200, seed=4, n_bins=8)
        sig1 = r.sigma.cpu().numpy()
        second = r.iterate(sites, 3, 200, seed=5, n_bins=8, keep_fields=True)
        _, wt, _ = _oracle_iteration(hop, eps, mu, U, beta, L, nf, sig1, sites, 3, 200, 5, 8)
        assert np.max(np.abs(second["weiss_tau"] - wt)) < 1e-12
        probs = [dict(L=L, beta=beta, U=U, weiss=wt[j], n_warmup=3, n_measure=200, recompute_every=50, n_bins=8,
                      seed=5, site=int(sites[j]), init_fields=first["results"][j]["fields"]) for j in range(12)]
        ref = oracle.run(probs, n_threads=8)
        for g, o in zip(second["results"], ref):
            assert np.array_equal(g["fields"], o["fields"])
            assert np.max(np.abs(g["bins"] - o["bins"])) < 1e-9
    finally:
        r.close()
