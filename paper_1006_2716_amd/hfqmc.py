"""ctypes binding of libhfqmc.so, the gfx950 Hirsch-Fye QMC engine.

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI declared in ``include/hfqmc.h``.  PyTorch provides device
memory (workspace and pool tensors) and the HIP stream.  There is no CPU
fallback: if the library is missing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhfqmc.so")

OK, EINVAL, ENOMEM, EDEVICE, EAGAIN, ENUMERIC, ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED = 0, 1
STATIC_BYTES = 64 << 20  # HFQMC_STATIC_BYTES: the device array of hfqmc_solve_static


class HFQMCError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hfqmc status {status}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [
        ("L", C.c_int32), ("beta", C.c_double), ("U", C.c_double),
        ("weiss", C.POINTER(C.c_double) * 2),
        ("n_warmup", C.c_int64), ("n_measure", C.c_int64),
        ("recompute_every", C.c_int32), ("n_bins", C.c_int32),
        ("seed", C.c_uint64), ("site_id", C.c_uint64), ("sweep_offset", C.c_int64),
        ("init_fields", C.POINTER(C.c_int8)), ("delay", C.c_int32), ("n_chains", C.c_int32),
    ]


class Result(C.Structure):
    _fields_ = [
        ("g", C.POINTER(C.c_double) * 2), ("g_err", C.POINTER(C.c_double) * 2),
        ("bins", C.POINTER(C.c_double)), ("final_fields", C.POINTER(C.c_int8)),
        ("n", C.c_double * 2), ("n_err", C.c_double * 2),
        ("docc", C.c_double), ("docc_err", C.c_double),
        ("accept_rate", C.c_double), ("max_drift", C.c_double),
        ("proposals", C.c_int64), ("accepts", C.c_int64), ("nonpositive", C.c_int64),
        ("status", C.c_int32), ("recoveries", C.c_int32),
    ]


class ServeStats(C.Structure):
    _fields_ = [
        ("submitted", C.c_int64), ("completed", C.c_int64), ("cancelled", C.c_int64), ("launches", C.c_int64),
        ("steps", C.c_int64),
        ("pending", C.c_int32), ("active", C.c_int32), ("capacity_used", C.c_double), ("capacity", C.c_double),
        ("step_ms_avg", C.c_double), ("launch_ms_avg", C.c_double),
    ]


_lib = None
_VP = C.c_void_p


def lib():
    """Load libhfqmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it with __graft_entry__.build() "
                               "(hipcc --offload-arch=gfx950); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        sig = {
            "hfqmc_lambda": [C.c_double, C.c_double, C.POINTER(C.c_double)],
            "hfqmc_create": [C.c_int, _VP, C.c_int, C.c_char_p, C.POINTER(_VP)],
            "hfqmc_workspace_size": [_VP, C.POINTER(Problem), C.c_int32, C.POINTER(C.c_size_t)],
            "hfqmc_solve": [_VP, C.POINTER(Problem), C.c_int32, _VP, C.c_size_t, C.POINTER(Result)],
            "hfqmc_solve_static": [_VP, C.POINTER(Problem), C.c_int32, C.POINTER(Result)],
            "hfqmc_set_drift_limit": [_VP, C.c_double],
            "hfqmc_debug_poison": [_VP, C.c_int64, C.c_int64],
            "hfqmc_stage": [_VP, C.POINTER(Problem), C.c_int32, _VP, C.c_size_t],
            "hfqmc_run": [_VP],
            "hfqmc_collect": [_VP, C.POINTER(Result)],
            "hfqmc_last_run_ms": [_VP, C.POINTER(C.c_double), C.POINTER(C.c_int32)],
            "hfqmc_attach_pool": [_VP, _VP, C.c_size_t],
            "hfqmc_site_bytes": [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)],
            "hfqmc_site_open": [_VP, C.c_int32, C.c_int32, C.c_int32, C.POINTER(_VP)],
            "hfqmc_site_close": [_VP, _VP],
            "hfqmc_site_define": [_VP, _VP, C.POINTER(Problem)],
            "hfqmc_site_set_fields": [_VP, _VP, C.POINTER(C.c_int8)],
            "hfqmc_site_force_flips": [_VP, _VP, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_double)],
            "hfqmc_site_get_green": [_VP, _VP, C.c_int32, C.POINTER(C.c_double)],
            "hfqmc_site_get_fields": [_VP, _VP, C.POINTER(C.c_int8)],
            "hfqmc_site_recompute": [_VP, _VP, C.POINTER(C.c_double)],
            "hfqmc_run_graph": [_VP],
            "hfqmc_last_launch_ms": [_VP, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int32)],
            "hfqmc_tune": [_VP, C.POINTER(Problem), C.c_int32, _VP, C.c_size_t, C.c_int32],
            "hfqmc_plan": [_VP, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                           C.POINTER(C.c_double)],
            "hfqmc_serve_config": [_VP, C.c_double, C.c_int64, C.c_double],
            "hfqmc_submit": [_VP, _VP, C.POINTER(Problem), C.POINTER(C.c_uint64)],
            "hfqmc_poll": [_VP, C.c_uint64, C.POINTER(Result)],
            "hfqmc_cancel": [_VP, C.c_uint64],
            "hfqmc_serve_stats": [_VP, C.POINTER(ServeStats)],
            "hfqmc_extrapolate": [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)],
            "hfqmc_entropy": [C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.POINTER(C.c_double), C.c_double, C.c_double, C.POINTER(C.c_double)],
            "hfqmc_lattice_bytes": [C.c_int32, C.c_int32, C.POINTER(C.c_size_t)],
            "hfqmc_lattice_create": [_VP, C.c_int32, C.c_int32, C.POINTER(C.c_double), _VP, C.c_size_t,
                                     C.POINTER(_VP)],
            "hfqmc_lattice_destroy": [_VP, _VP],
            "hfqmc_lattice_workspace": [_VP, C.c_int32, C.POINTER(C.c_size_t)],
            "hfqmc_lattice_green": [_VP, _VP, C.c_int32, C.c_double, C.c_double, _VP, _VP, _VP, _VP, C.c_size_t],
            "hfqmc_lattice_weiss": [_VP, _VP, C.c_int32, C.c_double, C.c_double, C.c_int32, _VP, _VP, _VP,
                                    C.POINTER(C.c_int32), C.c_int32, _VP, _VP],
            "hfqmc_lattice_sigma": [_VP, _VP, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32, _VP,
                                    C.POINTER(C.c_int32), C.c_int32, _VP, _VP, _VP, C.c_double, _VP],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.hfqmc_destroy.argtypes = [_VP]
        L.hfqmc_destroy.restype = None
        L.hfqmc_last_error.argtypes = [_VP]
        L.hfqmc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(status, what=""):
    if status != OK:
        msg = lib().hfqmc_last_error(None)
        raise HFQMCError(status, f"{what}: {msg.decode() if msg else ''}")


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def lam(dtau: float, U: float) -> float:
    out = C.c_double()
    _check(lib().hfqmc_lambda(dtau, U, C.byref(out)), "hfqmc_lambda")
    return out.value


def _struct_dtype(S):
    """numpy dtype with the field offsets of ctypes Structure S (pointers as
    uint64 addresses), for filling or reading arrays of S column-wise."""
    names, formats, offsets = [], [], []
    for name, ct in S._fields_:
        shape = ()
        if issubclass(ct, C.Array):
            shape, ct = (ct._length_,), ct._type_
        if issubclass(ct, C._Pointer):
            f = "<u8"
        else:
            f = {C.c_double: "<f8", C.c_int32: "<i4", C.c_int64: "<i8", C.c_uint64: "<u8"}[ct]
        names.append(name)
        formats.append((f, shape) if shape else f)
        offsets.append(getattr(S, name).offset)
    return np.dtype(dict(names=names, formats=formats, offsets=offsets, itemsize=C.sizeof(S)))


def _view(arr, dt):
    return np.frombuffer((C.c_char * C.sizeof(arr)).from_buffer(arr), dtype=dt)


def _addr(a):
    return a.__array_interface__["data"][0]


_U64 = (1 << 64) - 1  # seeds and site ids wrap to 64 bits, as a ctypes uint64 field does


class _Problems:
    """Marshals problem dicts into an array of Problem structs; the Weiss
    samples and initial fields of all problems are packed into one buffer
    each, which this object keeps alive."""

    _dt = None

    def __init__(self, problems):
        if _Problems._dt is None:
            _Problems._dt = _struct_dtype(Problem)
        n = len(problems)
        self.arr = (Problem * max(n, 1))()
        self.n = n
        if n == 0:
            self.keep = []
            return
        Ls = np.array([int(p["L"]) for p in problems], dtype=np.int64)
        ws = []
        for p, L in zip(problems, Ls.tolist()):
            w = np.asarray(p["weiss"], dtype=np.float64)
            if w.size != 2 * L:
                raise ValueError(f"weiss of {w.size} samples for L = {L} (need 2 x L)")
            ws.append(w.reshape(-1))
        weiss = np.concatenate(ws)
        w_off = np.concatenate([[0], np.cumsum(2 * Ls)[:-1]])
        inits = [p.get("init_fields") for p in problems]
        has = [k for k, f in enumerate(inits) if f is not None]
        init_buf = None
        v = _view(self.arr, self._dt)
        if has:
            parts = []
            for k in has:
                f = np.asarray(inits[k], dtype=np.int8).reshape(-1)
                if f.size != Ls[k]:
                    raise ValueError(f"init_fields of {f.size} entries for L = {int(Ls[k])}")
                parts.append(f)
            init_buf = np.concatenate(parts)
            i_off = np.concatenate([[0], np.cumsum(Ls[has])[:-1]])
            v["init_fields"][has] = _addr(init_buf) + i_off
        self.keep = [weiss, init_buf]
        base = _addr(weiss)
        v["L"] = Ls
        v["beta"] = [float(p["beta"]) for p in problems]
        v["U"] = [float(p["U"]) for p in problems]
        v["weiss"][:, 0] = base + 8 * w_off
        v["weiss"][:, 1] = base + 8 * (w_off + Ls)
        v["n_warmup"] = [int(p["n_warmup"]) for p in problems]
        v["n_measure"] = [int(p["n_measure"]) for p in problems]
        v["recompute_every"] = [int(p.get("recompute_every", 50)) for p in problems]
        v["n_bins"] = [int(p["n_bins"]) for p in problems]
        v["seed"] = [int(p["seed"]) & _U64 for p in problems]
        v["site_id"] = [int(p.get("site", i)) & _U64 for i, p in enumerate(problems)]
        v["sweep_offset"] = [int(p.get("sweep_offset", 0)) for p in problems]
        v["delay"] = [int(p.get("delay", 0)) for p in problems]
        v["n_chains"] = [int(p.get("n_chains", 0)) for p in problems]


class _Results:
    def __init__(self, problems):
        n = len(problems)
        self.arr = (Result * max(n, 1))()
        self.bufs = []
        for i, p in enumerate(problems):
            L = int(p["L"])
            g = np.zeros((2, L + 1))
            ge = np.zeros((2, L + 1))
            bins = np.zeros((int(p["n_bins"]), 2 * (L + 1) + 3))
            ff = np.zeros(L, dtype=np.int8)
            self.bufs.append((g, ge, bins, ff))
            r = self.arr[i]
            r.g[0] = g[0].ctypes.data_as(C.POINTER(C.c_double))
            r.g[1] = g[1].ctypes.data_as(C.POINTER(C.c_double))
            r.g_err[0] = ge[0].ctypes.data_as(C.POINTER(C.c_double))
            r.g_err[1] = ge[1].ctypes.data_as(C.POINTER(C.c_double))
            r.bins = _dp(bins)
            r.final_fields = ff.ctypes.data_as(C.POINTER(C.c_int8))

    def to_list(self):
        out = []
        for i, (g, ge, bins, ff) in enumerate(self.bufs):
            r = self.arr[i]
            out.append(dict(g_up=g[0].copy(), g_dn=g[1].copy(), g_up_err=ge[0].copy(), g_dn_err=ge[1].copy(),
                            bins=bins.copy(), fields=ff.copy(), n_up=r.n[0], n_dn=r.n[1], n_up_err=r.n_err[0],
                            n_dn_err=r.n_err[1], docc=r.docc, docc_err=r.docc_err, accept_rate=r.accept_rate,
                            max_drift=r.max_drift, proposals=r.proposals, accepts=r.accepts,
                            nonpositive=r.nonpositive, status=r.status, recoveries=r.recoveries))
        return out


def _torch():
    import torch  # noqa: PLC0415  (torch is only needed for device memory and streams)
    return torch


class Context:
    """A library context bound to a device and a HIP stream (torch's current one by default)."""

    def __init__(self, device: int = 0, stream=None, precision: int = FP64, tune_cache: str | None = None):
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.device = device
        self.stream = stream
        h = _VP()
        tc = None if tune_cache is None else os.fsencode(tune_cache)
        _check(lib().hfqmc_create(device, _VP(stream.cuda_stream), precision, tc, C.byref(h)), "hfqmc_create")
        self.h = h
        self._staged = None
        self._pool = None
        self._tickets = {}

    def close(self):
        if self.h:
            lib().hfqmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_drift_limit(self, limit: float):
        """hfqmc_set_drift_limit: recompute-interval control (0 = off)."""
        _check(lib().hfqmc_set_drift_limit(self.h, float(limit)), "hfqmc_set_drift_limit")

    def debug_poison(self, sweep_a: int = -1, sweep_b: int = -1):
        """hfqmc_debug_poison: NaN into G at the start of sweep_a's first
        attempt and of sweep_b's repeated attempt (-1: never)."""
        _check(lib().hfqmc_debug_poison(self.h, int(sweep_a), int(sweep_b)), "hfqmc_debug_poison")

    # ---------------------------------------------------------------- batch
    def workspace_size(self, problems) -> int:
        P = _Problems(problems)
        b = C.c_size_t()
        _check(lib().hfqmc_workspace_size(self.h, P.arr, P.n, C.byref(b)), "hfqmc_workspace_size")
        return b.value

    def alloc_workspace(self, problems):
        torch = _torch()
        return torch.empty(self.workspace_size(problems), dtype=torch.uint8, device=f"cuda:{self.device}")

    def solve(self, problems, workspace=None):
        if len(problems) == 0:  # the library's empty batch: nothing runs
            _check(lib().hfqmc_solve(self.h, None, 0, None, 0, None), "hfqmc_solve")
            return []
        self.stage(problems, workspace)
        self.run()
        return self.collect()

    def solve_static(self, problems):
        """hfqmc_solve_static: the batch on the library's own device array
        (no workspace, nothing allocated); raises HFQMCError(EINVAL) when the
        batch needs more than STATIC_BYTES."""
        P = _Problems(problems)
        R = _Results(problems)
        st = lib().hfqmc_solve_static(self.h, P.arr, P.n, R.arr)
        res = R.to_list()
        if st not in (OK, ENUMERIC):
            _check(st, "hfqmc_solve_static")
        self._staged = None
        return res

    def stage(self, problems, workspace=None):
        if workspace is None:
            workspace = self.alloc_workspace(problems)
        P = _Problems(problems)
        _check(lib().hfqmc_stage(self.h, P.arr, P.n, _VP(workspace.data_ptr()),
                                 workspace.numel() * workspace.element_size()), "hfqmc_stage")
        self._staged = (P, list(problems), workspace)

    def run(self):
        _check(lib().hfqmc_run(self.h), "hfqmc_run")

    def collect(self):
        P, problems, ws = self._staged
        R = _Results(problems)
        st = lib().hfqmc_collect(self.h, R.arr)
        res = R.to_list()
        if st not in (OK, ENUMERIC):
            _check(st, "hfqmc_collect")
        return res

    def run_graph(self):
        _check(lib().hfqmc_run_graph(self.h), "hfqmc_run_graph")

    def last_run_ms(self):
        ms = C.c_double()
        n = C.c_int32()
        _check(lib().hfqmc_last_run_ms(self.h, C.byref(ms), C.byref(n)), "hfqmc_last_run_ms")
        return ms.value, n.value

    def last_launch_ms(self, i: int = 0):
        """(ms, padded L, items) of class kernel i of the last eager run."""
        ms, lt, n = C.c_double(), C.c_int32(), C.c_int32()
        _check(lib().hfqmc_last_launch_ms(self.h, i, C.byref(ms), C.byref(lt), C.byref(n)), "hfqmc_last_launch_ms")
        return ms.value, lt.value, n.value

    # ---------------------------------------------------------------- tuning
    def tune(self, problems, sweeps: int = 64, workspace=None):
        if workspace is None:
            workspace = self.alloc_workspace(problems)
        P = _Problems(problems)
        _check(lib().hfqmc_tune(self.h, P.arr, P.n, _VP(workspace.data_ptr()),
                                workspace.numel() * workspace.element_size(), int(sweeps)), "hfqmc_tune")
        self._staged = None

    def plan(self, L: int, delay: int = 0):
        """(tile-rows per wave, delay depth, tuned proposals/s or 0)."""
        rt, k, rate = C.c_int32(), C.c_int32(), C.c_double()
        _check(lib().hfqmc_plan(self.h, L, delay, C.byref(rt), C.byref(k), C.byref(rate)), "hfqmc_plan")
        return rt.value, k.value, rate.value

    # ---------------------------------------------------------------- serving
    def serve_config(self, step_ms: float = 8.0, quantum_proposals: int = 0, capacity_cus: float = 0.0):
        _check(lib().hfqmc_serve_config(self.h, float(step_ms), int(quantum_proposals), float(capacity_cus)),
               "hfqmc_serve_config")

    def submit(self, site: "Site", problem) -> int | None:
        """Queue a request; returns its ticket, or None if not admissible now (EAGAIN)."""
        P = _Problems([problem])
        t = C.c_uint64()
        st = lib().hfqmc_submit(self.h, site.h, P.arr, C.byref(t))
        if st == EAGAIN:
            return None
        _check(st, "hfqmc_submit")
        self._tickets[t.value] = dict(problem)
        return t.value

    def poll(self, ticket: int):
        """Result dict once the request is done, else None."""
        prob = self._tickets.get(ticket)
        if prob is None:
            raise HFQMCError(ENOTFOUND, f"hfqmc_poll: unknown ticket {ticket}")
        R = _Results([prob])
        st = lib().hfqmc_poll(self.h, ticket, R.arr)
        if st == EAGAIN:
            return None
        del self._tickets[ticket]
        if st not in (OK, ENUMERIC):
            _check(st, "hfqmc_poll")
        return R.to_list()[0]

    def cancel(self, ticket: int):
        _check(lib().hfqmc_cancel(self.h, ticket), "hfqmc_cancel")
        self._tickets.pop(ticket, None)

    def serve_stats(self) -> dict:
        s = ServeStats()
        _check(lib().hfqmc_serve_stats(self.h, C.byref(s)), "hfqmc_serve_stats")
        return {k: getattr(s, k) for k, _ in ServeStats._fields_}

    # ---------------------------------------------------------------- sites
    def attach_pool(self, nbytes: int):
        torch = _torch()
        self._pool = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{self.device}")
        _check(lib().hfqmc_attach_pool(self.h, _VP(self._pool.data_ptr()), int(nbytes)), "hfqmc_attach_pool")
        return self._pool

    def site(self, L: int, n_bins: int = 32, n_chains: int = 1):
        return Site(self, L, n_bins, n_chains)


def site_bytes(L: int, n_bins: int = 32, n_chains: int = 1) -> int:
    b = C.c_size_t()
    _check(lib().hfqmc_site_bytes(L, n_bins, n_chains, C.byref(b)), "hfqmc_site_bytes")
    return b.value


class Site:
    """Device-resident impurity state (fields and Green matrices) in the context pool."""

    def __init__(self, ctx: Context, L: int, n_bins: int = 32, n_chains: int = 1):
        self.ctx = ctx
        self.L = L
        self.n_chains = n_chains
        h = _VP()
        _check(lib().hfqmc_site_open(ctx.h, L, n_bins, n_chains, C.byref(h)), "hfqmc_site_open")
        self.h = h

    def close(self):
        if self.h:
            _check(lib().hfqmc_site_close(self.ctx.h, self.h), "hfqmc_site_close")
            self.h = None

    def define(self, problem):
        P = _Problems([problem])
        _check(lib().hfqmc_site_define(self.ctx.h, self.h, P.arr), "hfqmc_site_define")

    def set_fields(self, fields):
        f = np.ascontiguousarray(fields, dtype=np.int8)
        _check(lib().hfqmc_site_set_fields(self.ctx.h, self.h, f.ctypes.data_as(C.POINTER(C.c_int8))),
               "hfqmc_site_set_fields")

    def force_flips(self, slices):
        s = np.ascontiguousarray(slices, dtype=np.int32)
        ratios = np.zeros(max(len(s), 1))
        _check(lib().hfqmc_site_force_flips(self.ctx.h, self.h, s.ctypes.data_as(C.POINTER(C.c_int32)), len(s),
                                            _dp(ratios)), "hfqmc_site_force_flips")
        return ratios[:len(s)]

    def green(self, spin: int) -> np.ndarray:
        out = np.zeros((self.L, self.L))
        _check(lib().hfqmc_site_get_green(self.ctx.h, self.h, spin, _dp(out)), "hfqmc_site_get_green")
        return out

    def fields(self) -> np.ndarray:
        out = np.zeros(self.L, dtype=np.int8)
        _check(lib().hfqmc_site_get_fields(self.ctx.h, self.h, out.ctypes.data_as(C.POINTER(C.c_int8))),
               "hfqmc_site_get_fields")
        return out

    def recompute(self) -> float:
        d = C.c_double()
        _check(lib().hfqmc_site_recompute(self.ctx.h, self.h, C.byref(d)), "hfqmc_site_recompute")
        return d.value


def extrapolate(dtau, value, err=None, order: int = 1):
    """dtau -> 0 fit value = sum_k c_k dtau^(2k): (c, c_err or None)."""
    d = np.ascontiguousarray(dtau, dtype=np.float64)
    v = np.ascontiguousarray(value, dtype=np.float64)
    e = None if err is None else np.ascontiguousarray(err, dtype=np.float64)
    c = np.zeros(order + 1)
    ce = np.zeros(order + 1)
    _check(lib().hfqmc_extrapolate(d.size, _dp(d), _dp(v), None if e is None else _dp(e), order, _dp(c), _dp(ce)),
           "hfqmc_extrapolate")
    return c, (None if e is None else ce)


def entropy(mu, n_lo, n_hi, T_lo: float, T_hi: float):
    """Per-site entropy s[k, i] from densities n_lo, n_hi (K, sites) at T_lo < T_hi
    on the ascending grid mu (K,), integrated from the empty system at mu[0]."""
    m = np.ascontiguousarray(mu, dtype=np.float64)
    a = np.ascontiguousarray(n_lo, dtype=np.float64)
    b = np.ascontiguousarray(n_hi, dtype=np.float64)
    if a.ndim != 2 or a.shape != b.shape or a.shape[0] != m.size:
        raise ValueError("entropy: need n_lo, n_hi of shape (len(mu), n_sites)")
    out = np.zeros_like(a)
    _check(lib().hfqmc_entropy(m.size, a.shape[1], _dp(m), _dp(a), _dp(b), T_lo, T_hi, _dp(out)), "hfqmc_entropy")
    return out


# ---------------------------------------------------------------- lattice
def _dev(t, dtype, shape, what):
    """Check a torch tensor argument: CUDA, contiguous, dtype and shape."""
    if not (t.is_cuda and t.is_contiguous() and t.dtype == dtype and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"{what}: need a contiguous {dtype} CUDA tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")
    return _VP(t.data_ptr())


class Lattice:
    """Layered lattice for the self-consistency calls (hopping blocks on the
    device).  Arrays are torch tensors on the context's device: eps float64
    (2, N), sigma / gloc complex128 (2, n_freq, N)."""

    def __init__(self, ctx: Context, hop, layer: int):
        torch = _torch()
        hop = np.ascontiguousarray(hop, dtype=np.float64)
        self.ctx = ctx
        self.n_sites = hop.shape[0]
        self.layer = int(layer)
        b = C.c_size_t()
        _check(lib().hfqmc_lattice_bytes(self.n_sites, self.layer, C.byref(b)), "hfqmc_lattice_bytes")
        self._mem = torch.empty(b.value, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        h = _VP()
        _check(lib().hfqmc_lattice_create(ctx.h, self.n_sites, self.layer, _dp(hop), _VP(self._mem.data_ptr()),
                                          b.value, C.byref(h)), "hfqmc_lattice_create")
        self.h = h
        self._ws = None

    def close(self):
        if self.h:
            _check(lib().hfqmc_lattice_destroy(self.ctx.h, self.h), "hfqmc_lattice_destroy")
            self.h = None

    def workspace_size(self, n_freq: int) -> int:
        b = C.c_size_t()
        _check(lib().hfqmc_lattice_workspace(self.h, n_freq, C.byref(b)), "hfqmc_lattice_workspace")
        return b.value

    def green(self, n_freq: int, beta: float, mu: float, eps, sigma, out=None):
        """Eq. (2): site-diagonal lattice Green function, complex128 (2, n_freq, N)."""
        torch = _torch()
        N = self.n_sites
        if out is None:
            out = torch.empty((2, n_freq, N), dtype=torch.complex128, device=sigma.device)
        need = self.workspace_size(n_freq)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=sigma.device)
        _check(lib().hfqmc_lattice_green(self.ctx.h, self.h, n_freq, beta, mu,
                                         _dev(eps, torch.float64, (2, N), "eps"),
                                         _dev(sigma, torch.complex128, (2, n_freq, N), "sigma"),
                                         _dev(out, torch.complex128, (2, n_freq, N), "gloc"),
                                         _VP(self._ws.data_ptr()), self._ws.numel()), "hfqmc_lattice_green")
        return out

    def weiss(self, n_freq: int, beta: float, mu: float, L: int, eps, gloc, sigma, sites):
        """Weiss functions of `sites`: (complex128 (2, n_freq, n_sel), float64 (n_sel, 2, L))."""
        torch = _torch()
        N = self.n_sites
        st = np.ascontiguousarray(sites, dtype=np.int32)
        n_sel = st.size
        w_iw = torch.empty((2, n_freq, n_sel), dtype=torch.complex128, device=gloc.device)
        w_tau = torch.empty((n_sel, 2, L), dtype=torch.float64, device=gloc.device)
        _check(lib().hfqmc_lattice_weiss(self.ctx.h, self.h, n_freq, beta, mu, L,
                                         _dev(eps, torch.float64, (2, N), "eps"),
                                         _dev(gloc, torch.complex128, (2, n_freq, N), "gloc"),
                                         _dev(sigma, torch.complex128, (2, n_freq, N), "sigma"),
                                         st.ctypes.data_as(C.POINTER(C.c_int32)), n_sel,
                                         _VP(w_iw.data_ptr()), _VP(w_tau.data_ptr())), "hfqmc_lattice_weiss")
        return w_iw, w_tau

    def sigma_update(self, n_freq: int, beta: float, mu: float, U: float, L: int, eps, sites, weiss_iw,
                     gimp_tau, density, mix: float, sigma):
        """sigma <- mix sigma_new + (1 - mix) sigma at `sites` (in place)."""
        torch = _torch()
        N = self.n_sites
        st = np.ascontiguousarray(sites, dtype=np.int32)
        n_sel = st.size
        _check(lib().hfqmc_lattice_sigma(self.ctx.h, self.h, n_freq, beta, mu, U, L,
                                         _dev(eps, torch.float64, (2, N), "eps"),
                                         st.ctypes.data_as(C.POINTER(C.c_int32)), n_sel,
                                         _dev(weiss_iw, torch.complex128, (2, n_freq, n_sel), "weiss_iw"),
                                         _dev(gimp_tau, torch.float64, (n_sel, 2, L + 1), "gimp_tau"),
                                         _dev(density, torch.float64, (n_sel, 2), "density"), mix,
                                         _dev(sigma, torch.complex128, (2, n_freq, N), "sigma")),
               "hfqmc_lattice_sigma")
        return sigma
