"""ctypes binding of the liblogdet C ABI (include/liblogdet.h).

Argument marshalling only: every step of an estimate runs in the HIP library.
The functions keep the C names; handles are opaque ctypes pointers.  A
missing or unloadable library raises immediately - there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "liblogdet.so")

LD_OK = 0
LD_PENDING = 1
LD_E_INVALID_ARG = -1
LD_E_BAD_CSR = -2
LD_E_NOT_SPD = -3
LD_E_NUMERIC = -4
LD_E_NO_MEMORY = -5
LD_E_BUSY = -6
LD_E_DEVICE = -7
LD_E_UNKNOWN_TICKET = -8

LD_VT_FP64, LD_VT_FP32, LD_VT_BF16 = 0, 1, 2
LD_METHOD_OSLQ, LD_METHOD_OSA_IOP, LD_METHOD_SO_SLQ = 0, 1, 2
LD_PROBE_RADEMACHER, LD_PROBE_GAUSSIAN = 0, 1
LD_PREC_FP64, LD_PREC_MIXED, LD_PREC_HALF, LD_PREC_AUTO = 0, 1, 2, 3

_STATUS_NAMES = {
    0: "LD_OK", 1: "LD_PENDING", -1: "LD_E_INVALID_ARG", -2: "LD_E_BAD_CSR",
    -3: "LD_E_NOT_SPD", -4: "LD_E_NUMERIC", -5: "LD_E_NO_MEMORY", -6: "LD_E_BUSY",
    -7: "LD_E_DEVICE", -8: "LD_E_UNKNOWN_TICKET",
}


class LdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class ld_ctx_opts(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_slots", C.c_int32),
                ("hbm_budget_bytes", C.c_uint64), ("hip_stream", C.c_void_p),
                ("default_method", C.c_int32), ("default_precision", C.c_int32)]


class ld_params(C.Structure):
    _fields_ = [("method", C.c_int32), ("precision", C.c_int32), ("n_probes", C.c_int32),
                ("sketch_rank", C.c_int32), ("krylov_steps", C.c_int32),
                ("iop_window", C.c_int32), ("seed", C.c_uint64), ("tol", C.c_double),
                ("probe_dist", C.c_int32), ("subspace_rank", C.c_int32),
                ("adapt_tol", C.c_double), ("adapt_every", C.c_int32),
                ("sketch_passes", C.c_int32)]


class ld_result(C.Structure):
    _fields_ = [("logdet", C.c_double), ("tr_sketch", C.c_double), ("tr_resid", C.c_double),
                ("shift_c", C.c_double), ("lambda_lo", C.c_double), ("lambda_hi", C.c_double),
                ("scale", C.c_double), ("probe_steps", C.c_int64), ("matvecs", C.c_int64),
                ("min_steps", C.c_int32), ("n_breakdowns", C.c_int32),
                ("device_ms", C.c_double), ("latency_ms", C.c_double),
                ("basis_rank", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ld_serving_stats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("ticks", C.c_uint64),
                ("batched_steps", C.c_uint64), ("batched_launches", C.c_uint64),
                ("held_bytes", C.c_uint64), ("peak_held_bytes", C.c_uint64),
                ("budget_bytes", C.c_uint64), ("buffer_allocs", C.c_uint64),
                ("buffer_frees", C.c_uint64), ("peak_active", C.c_int32),
                ("max_slots", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class ld_graph_stats(C.Structure):
    _fields_ = [("captures", C.c_uint64), ("replays", C.c_uint64), ("eager", C.c_uint64),
                ("cached", C.c_uint64), ("mode", C.c_int32),
                ("capture_failed", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int32)


class ld_detail(C.Structure):
    _fields_ = [("probe_K", _DP), ("probe_norm2", _DP), ("probe_steps", _IP),
                ("tri_alpha", _DP), ("tri_beta", _DP), ("sketch_basis", _DP)]


class ld_tune_result(C.Structure):
    _fields_ = [("spmm_lanes", C.c_int32), ("spmm_chunks", C.c_int32),
                ("update_lanes", C.c_int32), ("update_chunks", C.c_int32),
                ("spmm_ms", C.c_double), ("spmm_default_ms", C.c_double),
                ("update_ms", C.c_double), ("update_default_ms", C.c_double),
                ("candidates", C.c_int32), ("spmm_entry_split", C.c_int32),
                ("spmm_interleave", C.c_int32), ("spmm_row_stride", C.c_int32),
                ("step_presub", C.c_int32), ("step_presub_ms", C.c_double),
                ("step_plain_ms", C.c_double), ("spmm_row_groups", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib: Optional[C.CDLL] = None

# (name, restype, argtypes) of every function declared in include/liblogdet.h
_SIGNATURES = [
    ("ld_ctx_create", C.c_int32, [C.POINTER(ld_ctx_opts), C.POINTER(C.c_void_p)]),
    ("ld_ctx_destroy", C.c_int32, [C.c_void_p]),
    ("ld_last_error", C.c_char_p, []),
    ("ld_create_csr", C.c_int32, [C.c_void_p, C.c_int64, C.c_int64, _IP, _IP, _DP, C.c_int32,
                                  C.c_double, C.c_double, C.POINTER(C.c_void_p)]),
    ("ld_destroy", C.c_int32, [C.c_void_p]),
    ("ld_matrix_bounds", C.c_int32, [C.c_void_p, _DP, _DP]),
    ("ld_quad_form", C.c_int32, [C.c_void_p, _DP, _DP]),
    ("ld_autotune", C.c_int32, [C.c_void_p, C.POINTER(ld_params), C.c_int32,
                                C.POINTER(ld_tune_result)]),
    ("ld_tune_set", C.c_int32, [C.c_void_p, C.POINTER(ld_params), C.c_int32, C.c_int32,
                                C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                C.c_int32, C.c_int32]),
    ("ld_estimate", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                C.c_uint64, C.POINTER(ld_result)]),
    ("ld_estimate_ex", C.c_int32, [C.c_void_p, C.POINTER(ld_params), C.POINTER(ld_result)]),
    ("ld_request_bytes", C.c_int32, [C.c_void_p, C.POINTER(ld_params), C.POINTER(C.c_uint64)]),
    ("ld_estimate_detail", C.c_int32, [C.c_void_p, C.POINTER(ld_params), C.POINTER(ld_result),
                                       C.POINTER(ld_detail)]),
    ("ld_estimate_noalloc", C.c_int32, [C.c_void_p, C.POINTER(ld_params), C.POINTER(ld_result)]),
    ("ld_submit", C.c_int32, [C.c_void_p, C.POINTER(ld_params), C.POINTER(C.c_uint64)]),
    ("ld_serving_stats_get", C.c_int32, [C.c_void_p, C.POINTER(ld_serving_stats)]),
    ("ld_graph_mode", C.c_int32, [C.c_void_p, C.c_int32]),
    ("ld_graph_stats_get", C.c_int32, [C.c_void_p, C.POINTER(ld_graph_stats)]),
    ("ld_poll", C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(ld_result)]),
    ("ld_wait", C.c_int32, [C.c_void_p, C.c_uint64, C.POINTER(ld_result)]),
    ("ld_profile_enable", C.c_int32, [C.c_void_p, C.c_uint32]),
    ("ld_profile_query", C.c_int32, [C.c_void_p, C.c_uint32, C.POINTER(C.c_int64),
                                     C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("ld_debug_rademacher", C.c_int32, [C.c_void_p, C.c_uint64, C.c_int64, C.c_int32, C.c_int32,
                                        _DP]),
    ("ld_debug_copy", C.c_int32, [C.c_void_p, C.c_uint64, C.c_int32, _DP]),
    ("ld_debug_quad_log", C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, _DP, _DP, _IP,
                                      C.c_double, C.c_double, _DP, _IP]),
    ("ld_debug_stream", C.c_int32, [C.c_void_p, C.c_uint64, C.c_int32, C.c_int32, C.c_int32,
                                    _DP]),
    ("ld_debug_probes", C.c_int32, [C.c_void_p, C.c_uint64, C.c_int64, C.c_int32, C.c_int32,
                                    C.c_int32, _DP]),
    ("ld_debug_row_groups", C.c_int32, [C.c_void_p, C.POINTER(C.c_int64), _IP, _IP, _DP]),
]


def lib() -> C.CDLL:
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"liblogdet is not built ({LIB_PATH} missing): "
                              "run python -m paper_2606_07004_amd.build")
        handle = C.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def ld_last_error() -> str:
    msg = lib().ld_last_error()
    return msg.decode() if msg else ""


def _check(status: int) -> int:
    if status < 0:
        raise LdError(status, ld_last_error())
    return status


def ld_ctx_create(device: int = 0, max_slots: int = 0, hbm_budget_bytes: int = 0,
                  hip_stream=None, default_method: int = LD_METHOD_OSLQ,
                  default_precision: int = LD_PREC_FP64):
    """hip_stream: a raw hipStream_t (int) or an object with .cuda_stream (a
    torch.cuda.Stream), or None for a library-owned stream."""
    if hip_stream is not None and hasattr(hip_stream, "cuda_stream"):
        hip_stream = hip_stream.cuda_stream
    opts = ld_ctx_opts(device, max_slots, hbm_budget_bytes,
                       C.c_void_p(hip_stream) if hip_stream else None,
                       default_method, default_precision)
    out = C.c_void_p()
    _check(lib().ld_ctx_create(C.byref(opts), C.byref(out)))
    return out


def ld_ctx_destroy(ctx) -> None:
    _check(lib().ld_ctx_destroy(ctx))


def ld_create_csr(ctx, n: int, nnz: int, row_ptr, col_idx, values, vt: int = LD_VT_FP64,
                  lambda_lo_hint: float = 0.0, lambda_hi_hint: float = 0.0):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va = np.ascontiguousarray(values, dtype=np.float64)
    if rp.size != n + 1 or ci.size != nnz or va.size != nnz:
        raise LdError(LD_E_INVALID_ARG, "array sizes do not match n / nnz")
    out = C.c_void_p()
    _check(lib().ld_create_csr(ctx, n, nnz, rp.ctypes.data_as(_IP), ci.ctypes.data_as(_IP),
                               va.ctypes.data_as(_DP), vt, float(lambda_lo_hint),
                               float(lambda_hi_hint), C.byref(out)))
    return out


def ld_destroy(a) -> None:
    _check(lib().ld_destroy(a))


def ld_matrix_bounds(a):
    lo, hi = C.c_double(), C.c_double()
    _check(lib().ld_matrix_bounds(a, C.byref(lo), C.byref(hi)))
    return lo.value, hi.value


def make_params(n_probes: int, sketch_rank: int, krylov_steps: int, iop_window: int, seed: int,
                method: int = LD_METHOD_OSLQ, precision: int = LD_PREC_FP64,
                tol: float = 0.0, probe_dist: int = LD_PROBE_RADEMACHER,
                subspace_rank: int = 0, adapt_tol: float = 0.0,
                adapt_every: int = 0, sketch_passes: int = 0) -> ld_params:
    return ld_params(method, precision, n_probes, sketch_rank, krylov_steps, iop_window,
                     seed, tol, probe_dist, subspace_rank, adapt_tol, adapt_every, sketch_passes)


def runs_and_basis(params: ld_params):
    """(Krylov runs reported, basis columns) of a request, as ld_detail sizes them."""
    if params.method == LD_METHOD_SO_SLQ:
        k = params.subspace_rank if params.subspace_rank > 0 else min(10, params.sketch_rank)
        return k + params.n_probes - params.sketch_rank, k
    return params.n_probes, params.sketch_rank


def ld_estimate(a, n_probes: int, sketch_rank: int, krylov_steps: int, iop_window: int,
                seed: int) -> ld_result:
    res = ld_result()
    _check(lib().ld_estimate(a, n_probes, sketch_rank, krylov_steps, iop_window, seed,
                             C.byref(res)))
    return res


def ld_estimate_ex(a, params: ld_params) -> ld_result:
    res = ld_result()
    _check(lib().ld_estimate_ex(a, C.byref(params), C.byref(res)))
    return res


def ld_request_bytes(a, params: ld_params) -> int:
    """Device bytes an estimate with `params` takes beyond the matrix."""
    out = C.c_uint64()
    _check(lib().ld_request_bytes(a, C.byref(params), C.byref(out)))
    return out.value


def ld_estimate_noalloc(a, params: ld_params) -> ld_result:
    """ld_estimate_ex with the device buffers in the library's fixed scratch."""
    res = ld_result()
    _check(lib().ld_estimate_noalloc(a, C.byref(params), C.byref(res)))
    return res


def ld_estimate_detail(a, params: ld_params, n: Optional[int] = None, tri: bool = False,
                       basis: bool = False):
    """Estimate plus per-run arrays: dict with probe_K, probe_norm2,
    probe_steps and optionally tri_alpha/tri_beta ([runs, m]) and the sketch
    basis ([n, b])."""
    B, s = runs_and_basis(params)
    m = params.krylov_steps
    arrays = {"probe_K": np.zeros(B), "probe_norm2": np.zeros(B),
              "probe_steps": np.zeros(B, dtype=np.int32)}
    if tri:
        arrays["tri_alpha"] = np.zeros((B, m))
        arrays["tri_beta"] = np.zeros((B, m))
    if basis:
        if n is None:
            raise ValueError("n is needed to receive the sketch basis")
        arrays["sketch_basis"] = np.zeros((n, s))
    det = ld_detail()
    for name, arr in arrays.items():
        ptr_t = _IP if arr.dtype == np.int32 else _DP
        setattr(det, name, arr.ctypes.data_as(ptr_t))
    res = ld_result()
    _check(lib().ld_estimate_detail(a, C.byref(params), C.byref(res), C.byref(det)))
    return res, arrays


def ld_quad_form(a, x) -> float:
    """x^T Q x on the device (FP64)."""
    xv = np.ascontiguousarray(x, dtype=np.float64)
    out = C.c_double()
    _check(lib().ld_quad_form(a, xv.ctypes.data_as(_DP), C.byref(out)))
    return out.value


def ld_autotune(a, params: ld_params, reps: int = 20) -> ld_tune_result:
    """Time the Krylov-step kernel geometries on matrix `a` for the shapes of
    `params` and store the fastest in the matrix (reps = 0: drop it)."""
    out = ld_tune_result()
    _check(lib().ld_autotune(a, C.byref(params), int(reps), C.byref(out)))
    return out


def ld_tune_set(a, params: ld_params, spmm_lanes: int, spmm_chunks: int, update_lanes: int,
                update_chunks: int, spmm_entry_split: int = 1, spmm_interleave: int = 0,
                spmm_row_stride: int = 0, step_presub: int = 1, spmm_row_groups: int = 0) -> None:
    """Store a given product / update geometry for the estimate block of `params`."""
    _check(lib().ld_tune_set(a, C.byref(params), int(spmm_lanes), int(spmm_chunks),
                             int(spmm_entry_split), int(update_lanes), int(update_chunks),
                             int(spmm_interleave), int(spmm_row_stride), int(step_presub),
                             int(spmm_row_groups)))


def ld_serving_stats_get(ctx) -> ld_serving_stats:
    out = ld_serving_stats()
    _check(lib().ld_serving_stats_get(ctx, C.byref(out)))
    return out


def ld_graph_mode(ctx, mode: int) -> None:
    _check(lib().ld_graph_mode(ctx, int(mode)))


def ld_graph_stats_get(ctx) -> ld_graph_stats:
    out = ld_graph_stats()
    _check(lib().ld_graph_stats_get(ctx, C.byref(out)))
    return out


def ld_submit(a, params: ld_params) -> int:
    t = C.c_uint64()
    _check(lib().ld_submit(a, C.byref(params), C.byref(t)))
    return t.value


def ld_poll(ctx, ticket: int) -> Optional[ld_result]:
    """The result once the request has finished, None while it runs."""
    res = ld_result()
    st = _check(lib().ld_poll(ctx, ticket, C.byref(res)))
    return None if st == LD_PENDING else res


def ld_wait(ctx, ticket: int) -> ld_result:
    res = ld_result()
    _check(lib().ld_wait(ctx, ticket, C.byref(res)))
    return res


LD_PROF_SPMM, LD_PROF_DOTS, LD_PROF_UPDATE, LD_PROF_REDUCE = 1, 2, 4, 8
LD_PROF_SMALL, LD_PROF_SKETCH, LD_PROF_PROBES, LD_PROF_ALL = 16, 32, 64, 127
PROF_FAMILIES = {"spmm": 1, "dots": 2, "update": 4, "reduce": 8, "small": 16, "sketch": 32,
                 "probes": 64}


def ld_profile_enable(ctx, family_mask: int) -> None:
    _check(lib().ld_profile_enable(ctx, family_mask))


def ld_profile_query(ctx, family: int):
    """(launches, total_ms, total_algorithmic_bytes) summed over `family`."""
    n, ms, by = C.c_int64(), C.c_double(), C.c_double()
    _check(lib().ld_profile_query(ctx, family, C.byref(n), C.byref(ms), C.byref(by)))
    return n.value, ms.value, by.value


def ld_debug_rademacher(ctx, seed: int, n: int, col_begin: int, col_end: int) -> np.ndarray:
    out = np.zeros((n, col_end - col_begin))
    _check(lib().ld_debug_rademacher(ctx, seed, n, col_begin, col_end, out.ctypes.data_as(_DP)))
    return out


def ld_debug_probes(ctx, seed: int, n: int, col_begin: int, col_end: int,
                    dist: int = LD_PROBE_RADEMACHER) -> np.ndarray:
    out = np.zeros((n, col_end - col_begin))
    _check(lib().ld_debug_probes(ctx, seed, n, col_begin, col_end, dist,
                                 out.ctypes.data_as(_DP)))
    return out


def ld_debug_quad_log(ctx, alpha, beta, dims, a: float, b: float):
    """(K, need) of the tridiagonals (alpha[runs, m], beta[runs, m], dims[runs])
    by the estimates' quadrature kernels."""
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    be = np.ascontiguousarray(beta, dtype=np.float64)
    dm = np.ascontiguousarray(dims, dtype=np.int32)
    runs, m = al.shape
    assert be.shape == (runs, m) and dm.shape == (runs,)
    K = np.zeros(runs)
    need = np.zeros(runs, dtype=np.int32)
    _check(lib().ld_debug_quad_log(ctx, runs, m, al.ctypes.data_as(_DP), be.ctypes.data_as(_DP),
                                   dm.ctypes.data_as(_IP), float(a), float(b),
                                   K.ctypes.data_as(_DP), need.ctypes.data_as(_IP)))
    return K, need


def ld_debug_copy(ctx, nbytes: int, reps: int = 10) -> float:
    """Mean device ms of a plain copy of nbytes (calibration hook)."""
    ms = C.c_double()
    _check(lib().ld_debug_copy(ctx, nbytes, reps, C.byref(ms)))
    return ms.value


def ld_debug_stream(ctx, nbytes: int, reads: int, writes: int, reps: int = 10) -> float:
    """Mean device ms of a streaming kernel reading `reads` buffers of nbytes
    and writing `writes` (0 or 1) (attainable-bandwidth hook)."""
    ms = C.c_double()
    _check(lib().ld_debug_stream(ctx, nbytes, reads, writes, reps, C.byref(ms)))
    return ms.value


def ld_debug_row_groups(a, n: int):
    """The row groups matrix `a` (n rows) keeps: None, or (gp, col, val) with
    val of shape [union columns][4] (FP64)."""
    nu = C.c_int64()
    _check(lib().ld_debug_row_groups(a, C.byref(nu), None, None, None))
    if nu.value == 0:
        return None
    gp = np.zeros((n + 3) // 4 + 1, dtype=np.int32)
    col = np.zeros(nu.value, dtype=np.int32)
    val = np.zeros((nu.value, 4), dtype=np.float64)
    _check(lib().ld_debug_row_groups(a, C.byref(nu), gp.ctypes.data_as(_IP),
                                     col.ctypes.data_as(_IP), val.ctypes.data_as(_DP)))
    return gp, col, val


class Context:
    """Owning wrapper: a context plus the matrices created in it."""

    def __init__(self, device: int = 0, **kw):
        self.handle = ld_ctx_create(device, **kw)
        self._mats = []

    def matrix(self, csr, vt: int = LD_VT_FP64, lo_hint: float = 0.0, hi_hint: float = 0.0):
        h = ld_create_csr(self.handle, csr.n, csr.nnz, csr.row_ptr, csr.col_idx, csr.values,
                          vt, lo_hint, hi_hint)
        self._mats.append(h)
        return h

    def release(self, a) -> None:
        ld_destroy(a)
        self._mats = [m for m in self._mats if m.value != a.value]

    def close(self) -> None:
        for h in self._mats:
            ld_destroy(h)
        self._mats = []
        if self.handle is not None:
            ld_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
