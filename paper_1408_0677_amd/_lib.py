"""Loader of the in-tree HIP library (libmls_hip.so) and its C signatures.

There is no fallback: if the library has not been built, or cannot be
loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# MLS_HIP_LIB may name another build of the same sources (used to compare
# kernel variants); by default the in-tree library is loaded.
LIB_PATH = os.environ.get("MLS_HIP_LIB") or os.path.join(HERE, "libmls_hip.so")

# Symbols declared in include/mls.h.
CONTOUR_STATIC_SCRATCH_BYTES = 16 << 20   # MLS_CONTOUR_STATIC_SCRATCH_BYTES
EXPORTS = ("mls_status_string", "mls_last_error", "mls_context_create",
           "mls_context_destroy", "mls_fit", "mls_contour", "mls_fit_scratch_bytes",
           "mls_context_reserve", "mls_server_create", "mls_server_destroy",
           "mls_server_put_points", "mls_server_release_points", "mls_server_submit",
           "mls_server_poll", "mls_server_wait", "mls_server_last_error",
           "mls_server_tuning", "mls_server_tuned_classes", "mls_fit_grad", "mls_layout",
           "mls_contour_static", "mls_context_trace", "mls_context_trace_last",
           "mls_map_bands", "mls_map_adaptive", "mls_server_cancel",
           "mls_server_tuning_pending")


class MlsGrid(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class MlsWeight(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("h", ctypes.c_double),
                ("alpha", ctypes.c_double)]


class MlsSolveOpts(ctypes.Structure):
    _fields_ = [("pivot_tol", ctypes.c_double), ("weight_floor", ctypes.c_double),
                ("lp_terms", ctypes.c_int32), ("lp_slab", ctypes.c_int32),
                ("lp_form", ctypes.c_int32)]


class MlsLayoutParams(ctypes.Structure):
    _fields_ = [("C", ctypes.c_double), ("D", ctypes.c_double), ("eta", ctypes.c_double),
                ("t0", ctypes.c_double), ("lam", ctypes.c_double)]


class MlsAdaptiveParams(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("halfwidth", ctypes.c_double),
                ("fade_lo", ctypes.c_double), ("fade_hi", ctypes.c_double)]


class MlsRequest(ctypes.Structure):
    _fields_ = [("pointset", ctypes.c_uint64), ("basis", ctypes.c_int32),
                ("weight", MlsWeight), ("grid", MlsGrid), ("precision", ctypes.c_int32),
                ("opts", MlsSolveOpts), ("d_fields", ctypes.c_void_p),
                ("d_degree", ctypes.c_void_p), ("timeout_s", ctypes.c_double)]


class MlsResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_start", ctypes.c_double),
                ("t_end", ctypes.c_double), ("detail", ctypes.c_char * 128)]


TRACE_MAX_STAGES = 4   # MLS_TRACE_MAX_STAGES


class MlsTraceRecord(ctypes.Structure):
    _fields_ = [("call", ctypes.c_char * 16), ("form", ctypes.c_int32),
                ("n_stages", ctypes.c_int32),
                ("stage", (ctypes.c_char * 16) * TRACE_MAX_STAGES),
                ("ms", ctypes.c_double * TRACE_MAX_STAGES), ("total_ms", ctypes.c_double)]


_lib = None


def load():
    """Load libmls_hip.so (raises if it is missing or broken)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is not built; run paper_1408_0677_amd/build.py "
            "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.mls_status_string.argtypes = [ctypes.c_int]
    lib.mls_status_string.restype = ctypes.c_char_p
    lib.mls_last_error.argtypes = []
    lib.mls_last_error.restype = ctypes.c_char_p
    lib.mls_context_create.argtypes = [i32, ctypes.POINTER(P)]
    lib.mls_context_create.restype = ctypes.c_int
    lib.mls_context_destroy.argtypes = [P]
    lib.mls_context_destroy.restype = None
    lib.mls_fit.argtypes = [P, P, P, i64, i32, i32, ctypes.POINTER(MlsWeight),
                            ctypes.POINTER(MlsGrid), i32,
                            ctypes.POINTER(MlsSolveOpts), P, P, P]
    lib.mls_fit.restype = ctypes.c_int
    lib.mls_fit_grad.argtypes = [P, P, P, i64, i32, i32, ctypes.POINTER(MlsWeight),
                                 ctypes.POINTER(MlsGrid), i32, ctypes.POINTER(MlsSolveOpts),
                                 P, P, P, P]
    lib.mls_fit_grad.restype = ctypes.c_int
    lib.mls_layout.argtypes = [P, P, i64, P, P, i64, P, P, i64,
                               ctypes.POINTER(MlsLayoutParams), i32, P]
    lib.mls_layout.restype = ctypes.c_int
    lib.mls_contour.argtypes = [P, P, i32, ctypes.POINTER(MlsGrid), P, i32, P, P, P, i64,
                                ctypes.POINTER(i64), P]
    lib.mls_contour.restype = ctypes.c_int
    lib.mls_contour_static.argtypes = [P, P, i32, ctypes.POINTER(MlsGrid), P, i32, P, P, P,
                                       i64, P, P]
    lib.mls_contour_static.restype = ctypes.c_int
    lib.mls_fit_scratch_bytes.argtypes = [i64, i32, i32, ctypes.POINTER(MlsWeight),
                                          ctypes.POINTER(MlsGrid)]
    lib.mls_fit_scratch_bytes.restype = ctypes.c_size_t
    lib.mls_map_bands.argtypes = [P, P, i32, ctypes.POINTER(MlsGrid), P, i32, P, P, P, P]
    lib.mls_map_bands.restype = ctypes.c_int
    lib.mls_map_adaptive.argtypes = [P, P, P, i32, ctypes.POINTER(MlsGrid), P,
                                     ctypes.POINTER(MlsAdaptiveParams), P, P]
    lib.mls_map_adaptive.restype = ctypes.c_int
    lib.mls_context_trace.argtypes = [P, i32, ctypes.c_char_p]
    lib.mls_context_trace.restype = ctypes.c_int
    lib.mls_context_trace_last.argtypes = [P, ctypes.POINTER(MlsTraceRecord)]
    lib.mls_context_trace_last.restype = ctypes.c_int
    lib.mls_context_reserve.argtypes = [P, ctypes.c_size_t]
    lib.mls_context_reserve.restype = ctypes.c_int
    lib.mls_server_create.argtypes = [i32, ctypes.c_size_t, i32, ctypes.c_size_t,
                                      ctypes.POINTER(P)]
    lib.mls_server_create.restype = ctypes.c_int
    lib.mls_server_destroy.argtypes = [P]
    lib.mls_server_destroy.restype = None
    lib.mls_server_put_points.argtypes = [P, P, P, i64, i32, ctypes.POINTER(ctypes.c_uint64)]
    lib.mls_server_put_points.restype = ctypes.c_int
    lib.mls_server_release_points.argtypes = [P, ctypes.c_uint64]
    lib.mls_server_release_points.restype = ctypes.c_int
    lib.mls_server_submit.argtypes = [P, ctypes.POINTER(MlsRequest),
                                      ctypes.POINTER(ctypes.c_uint64)]
    lib.mls_server_submit.restype = ctypes.c_int
    lib.mls_server_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(MlsResult)]
    lib.mls_server_poll.restype = ctypes.c_int
    lib.mls_server_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(MlsResult)]
    lib.mls_server_wait.restype = ctypes.c_int
    lib.mls_server_last_error.argtypes = []
    lib.mls_server_last_error.restype = ctypes.c_char_p
    lib.mls_server_tuning.argtypes = [P, i32, ctypes.c_char_p]
    lib.mls_server_tuning.restype = ctypes.c_int
    lib.mls_server_tuned_classes.argtypes = [P]
    lib.mls_server_tuned_classes.restype = ctypes.c_int64
    lib.mls_server_tuning_pending.argtypes = [P]
    lib.mls_server_tuning_pending.restype = ctypes.c_int64
    lib.mls_server_cancel.argtypes = [P, ctypes.c_uint64]
    lib.mls_server_cancel.restype = ctypes.c_int
    _lib = lib
    return lib
