"""Plain CPU oracle for the Hirsch-Fye QMC impurity solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
module; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may use it.  It shares no code with the HIP library.

Contents
  * ``hfqmc_ref.c``   -- the Markov chain itself (plain loops, fp64, LU with
    partial pivoting for the Dyson equation, Sherman-Morrison updates), exposed
    through ctypes by the wrappers below;
  * ``exact.py``      -- exact results the chain must reproduce: enumeration of
    all 2^L Ising fields, the isolated atom, the BSS (determinantal) form of the
    same discrete problem and exact diagonalisation of a two-site Anderson
    model.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hfqmc_ref.c")
_LIB = os.path.join(_HERE, "libhfqmc_ref.so")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no fast-math) into oracle/."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
             _SRC, "-o", tmp, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [
        ("L", C.c_int32), ("beta", C.c_double), ("U", C.c_double),
        ("weiss_up", C.POINTER(C.c_double)), ("weiss_dn", C.POINTER(C.c_double)),
        ("n_warmup", C.c_int64), ("n_measure", C.c_int64),
        ("recompute_every", C.c_int32), ("n_bins", C.c_int32),
        ("seed", C.c_uint64), ("site", C.c_uint64), ("sweep_offset", C.c_int64),
        ("init_fields", C.POINTER(C.c_int8)), ("chain", C.c_uint64),
    ]


class _Result(C.Structure):
    _fields_ = [
        ("bins", C.POINTER(C.c_double)), ("final_fields", C.POINTER(C.c_int8)),
        ("final_green", C.POINTER(C.c_double)),
        ("proposals", C.c_int64), ("accepts", C.c_int64), ("nonpositive", C.c_int64),
        ("max_drift", C.c_double), ("status", C.c_int32),
        ("hist", C.POINTER(C.c_int64)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = C.CDLL(_LIB)
        L.ref_lambda.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double)]
        L.ref_philox4x64.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
        L.ref_weiss_matrix.argtypes = [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ref_dyson.argtypes = [C.c_int, C.POINTER(C.c_double), C.c_double, C.c_int,
                                C.POINTER(C.c_int8), C.POINTER(C.c_double)]
        L.ref_force_flips.argtypes = [C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                                      C.POINTER(C.c_int8), C.POINTER(C.c_int32), C.c_int,
                                      C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ref_run.argtypes = [C.POINTER(_Problem), C.c_int, C.POINTER(_Result), C.c_int]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lam(dtau: float, U: float) -> float:
    out = C.c_double()
    if lib().ref_lambda(dtau, U, C.byref(out)) != 0:
        raise ValueError("invalid dtau/U")
    return out.value


def philox4x64(ctr, key) -> np.ndarray:
    c = (C.c_uint64 * 4)(*[int(v) for v in ctr])
    k = (C.c_uint64 * 2)(*[int(v) for v in key])
    o = (C.c_uint64 * 4)()
    lib().ref_philox4x64(c, k, o)
    return np.array(list(o), dtype=np.uint64)


def weiss_matrix(g: np.ndarray) -> np.ndarray:
    g = np.ascontiguousarray(g, dtype=np.float64)
    L = g.shape[0]
    out = np.empty((L, L))
    lib().ref_weiss_matrix(L, _dp(g), _dp(out))
    return out


def dyson(g: np.ndarray, lam_: float, sigma: int, s: np.ndarray) -> np.ndarray:
    g = np.ascontiguousarray(g, dtype=np.float64)
    s = np.ascontiguousarray(s, dtype=np.int8)
    L = g.shape[0]
    G = np.empty((L, L))
    rc = lib().ref_dyson(L, _dp(g), lam_, sigma, s.ctypes.data_as(C.POINTER(C.c_int8)), _dp(G))
    if rc:
        raise RuntimeError(f"ref_dyson failed: {rc}")
    return G


def force_flips(g_up, g_dn, lam_, s, slices):
    """Dyson(s) followed by forced Sherman-Morrison flips of `slices`.

    Returns (G_up, G_dn, final_fields, ratios)."""
    g_up = np.ascontiguousarray(g_up, dtype=np.float64)
    g_dn = np.ascontiguousarray(g_dn, dtype=np.float64)
    s = np.array(s, dtype=np.int8, copy=True)
    sl = np.ascontiguousarray(slices, dtype=np.int32)
    L = g_up.shape[0]
    Gu = np.empty((L, L)); Gd = np.empty((L, L)); rat = np.empty(max(len(sl), 1))
    rc = lib().ref_force_flips(L, _dp(g_up), _dp(g_dn), lam_, s.ctypes.data_as(C.POINTER(C.c_int8)),
                               sl.ctypes.data_as(C.POINTER(C.c_int32)), len(sl), _dp(Gu), _dp(Gd), _dp(rat))
    if rc:
        raise RuntimeError(f"ref_force_flips failed: {rc}")
    return Gu, Gd, s, rat[:len(sl)]


def n_values(L: int) -> int:
    """Number of measured values per bin: g_up(0..L), g_dn(0..L), n_up, n_dn, d."""
    return 2 * (L + 1) + 3


def run(problems, n_threads: int = 1, want_green: bool = False, want_hist: bool = False):
    """Run one Markov chain per problem dict.

    Problem keys: L, beta, U, weiss (2 x L array), n_warmup, n_measure,
    recompute_every, n_bins, seed, site, [sweep_offset], [init_fields],
    [chain] (Philox counter word 3; independent chains of one impurity).
    Returns a list of dicts with 'bins' (n_bins x NV), 'fields', 'green',
    'proposals', 'accepts', 'nonpositive', 'max_drift', 'status'.
    """
    n = len(problems)
    P = (_Problem * max(n, 1))()
    R = (_Result * max(n, 1))()
    keep = []
    outs = []
    for i, p in enumerate(problems):
        L = int(p["L"])
        w = np.ascontiguousarray(p["weiss"], dtype=np.float64).reshape(2, L)
        wu = np.ascontiguousarray(w[0]); wd = np.ascontiguousarray(w[1])
        bins = np.zeros((int(p["n_bins"]), n_values(L)))
        fields = np.zeros(L, dtype=np.int8)
        green = np.zeros((2, L, L)) if want_green else None
        hist = np.zeros(1 << L, dtype=np.int64) if (want_hist and L <= 20) else None
        init = p.get("init_fields")
        init_arr = None if init is None else np.ascontiguousarray(init, dtype=np.int8)
        keep += [wu, wd, bins, fields, green, init_arr, hist]
        P[i] = _Problem(L, float(p["beta"]), float(p["U"]), _dp(wu), _dp(wd),
                        int(p["n_warmup"]), int(p["n_measure"]), int(p.get("recompute_every", 50)),
                        int(p["n_bins"]), int(p["seed"]), int(p.get("site", i)),
                        int(p.get("sweep_offset", 0)),
                        None if init_arr is None else init_arr.ctypes.data_as(C.POINTER(C.c_int8)),
                        int(p.get("chain", 0)))
        R[i].bins = _dp(bins)
        R[i].final_fields = fields.ctypes.data_as(C.POINTER(C.c_int8))
        R[i].final_green = _dp(green) if green is not None else None
        R[i].hist = hist.ctypes.data_as(C.POINTER(C.c_int64)) if hist is not None else None
        outs.append((bins, fields, green, hist))
    lib().ref_run(P, n, R, int(n_threads))
    res = []
    for i in range(n):
        bins, fields, green, hist = outs[i]
        res.append(dict(bins=bins, fields=fields, green=green, hist=hist, proposals=R[i].proposals,
                        accepts=R[i].accepts, nonpositive=R[i].nonpositive,
                        max_drift=R[i].max_drift, status=R[i].status))
    return res


def summarize(bins: np.ndarray, L: int):
    """Bin means -> (values, errors) with errors = std(ddof=1)/sqrt(n_bins)."""
    nb = bins.shape[0]
    mean = bins.mean(axis=0)
    err = bins.std(axis=0, ddof=1) / np.sqrt(nb)
    return dict(
        g_up=mean[0:L + 1], g_dn=mean[L + 1:2 * L + 2],
        g_up_err=err[0:L + 1], g_dn_err=err[L + 1:2 * L + 2],
        n_up=mean[2 * L + 2], n_dn=mean[2 * L + 3], docc=mean[2 * L + 4],
        n_up_err=err[2 * L + 2], n_dn_err=err[2 * L + 3], docc_err=err[2 * L + 4])


def run_chains(problem, n_chains: int, n_threads: int = 1):
    """Several independent chains of one impurity: chain j draws with
    counter word 3 = j, runs the full warm-up and n_measure // n_chains
    measured sweeps (the first n_measure % n_chains chains one more), and the
    bins of the chains are pooled: bin b of the result is the mean over all
    chains' measurements that fall in their bin b.  Returns the pooled bin
    means, the per-bin measurement counts and the per-chain results."""
    nm = int(problem["n_measure"])
    nb = int(problem["n_bins"])
    parts = [dict(problem, chain=j, n_measure=nm // n_chains + (1 if j < nm % n_chains else 0))
             for j in range(n_chains)]
    res = run(parts, n_threads=n_threads)
    NV = res[0]["bins"].shape[1]
    sums = np.zeros((nb, NV))
    counts = np.zeros(nb)
    for part, r in zip(parts, res):
        m = np.arange(part["n_measure"])
        cnt = np.bincount((m * nb) // part["n_measure"], minlength=nb).astype(float)
        sums += r["bins"] * cnt[:, None]
        counts += cnt
    return sums / counts[:, None], counts, res
