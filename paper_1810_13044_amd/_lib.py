"""ctypes binding of libslk (include/slk.h).  Argument marshalling only: every step of
the computation runs in the library's HIP kernels.  Device arrays are torch tensors on
the current HIP device; the current torch stream is passed to the library."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libslk.so")

SLK_OK = 0
STATUS = {0: "SLK_OK", 1: "SLK_ERR_INVALID_ARG", 2: "SLK_ERR_OUT_OF_MEMORY", 3: "SLK_ERR_DEVICE",
          4: "SLK_ERR_NUMERIC", 5: "SLK_ERR_UNSUPPORTED"}
PREC_FP32, PREC_BF16, PREC_BF16X = 0, 1, 2
KNN_AUTO, KNN_EXACT, KNN_MFMA = 0, 1, 2


class SlkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class KnnOpts(C.Structure):
    _fields_ = [("k", C.c_int32), ("reorder", C.c_int32), ("candidates", C.c_int32),
                ("method", C.c_int32), ("prec", C.c_int32)]


class GraphInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("k", C.c_int32), ("reordered", C.c_int32), ("nnz", C.c_int64),
                ("max_degree", C.c_int32), ("min_degree", C.c_int32), ("sigma2", C.c_double),
                ("rows_certified", C.c_int64), ("rows_fallback", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("sigma2", C.c_double), ("delta", C.c_double),
                ("bound_tol", C.c_double), ("max_outer", C.c_int32), ("max_inner", C.c_int32),
                ("fixed_inner", C.c_int32), ("pairwise_scale", C.c_int32), ("prec", C.c_int32),
                ("final_pass", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("inner_iters_total", C.c_int32),
                ("inner_iters_last", C.c_int32), ("converged", C.c_int32),
                ("n_distinct_modes", C.c_int32), ("final_passes", C.c_int32), ("energy", C.c_double),
                ("energy_fp64", C.c_double), ("bound", C.c_double), ("cut", C.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class EnergyOut(C.Structure):
    _fields_ = [("energy", C.c_double), ("energy_fp64", C.c_double), ("bound", C.c_double),
                ("cut", C.c_int64)]


class Job(C.Structure):
    _fields_ = [("x", C.c_void_p), ("n", C.c_int64), ("d", C.c_int32), ("L", C.c_int32),
                ("init_modes_host", C.c_void_p), ("knn", KnnOpts), ("params", Params),
                ("z_out", C.c_void_p), ("labels_out", C.c_void_p), ("modes_out_host", C.c_void_p),
                ("result_host", C.c_void_p), ("status_host", C.c_void_p)]


class ServerOpts(C.Structure):
    _fields_ = [("max_jobs", C.c_int32), ("passes_per_step", C.c_int32), ("memory_budget", C.c_int64),
                ("builders", C.c_int32), ("graph_replay", C.c_int32)]


class TuneParams(C.Structure):
    _fields_ = [("wave_steps", C.c_int32), ("knn_exact_width", C.c_int32), ("knn_exact", C.c_int32),
                ("knn_long_scan", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("graph_launches", C.c_int64), ("graph_captures", C.c_int64),
                ("grouped_builds", C.c_int64)]


class KnnItem(C.Structure):
    _fields_ = [("x", C.c_void_p), ("n", C.c_int64), ("d", C.c_int32), ("reserved", C.c_int32), ("opts", KnnOpts)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libslk.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libslk.so not found at {path}: run `python -m paper_1810_13044_amd.build`")
    lib = C.CDLL(path)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "slk_knn_opts_default": [C.POINTER(KnnOpts)],
        "slk_build_knn": [P, I64, I32, C.POINTER(KnnOpts), P, C.POINTER(P)],
        "slk_graph_from_knn": [I64, I32, P, P, I32, P, C.POINTER(P)],
        "slk_graph_from_csr": [I64, I64, P, P, D, I32, P, C.POINTER(P)],
        "slk_graph_info": [P, C.POINTER(GraphInfo)],
        "slk_graph_export": [P, P, P, P, P, P, P],
        "slk_params_default": [C.POINTER(Params)],
        "slk_assign": [P, I64, I32, P, I32, P, C.POINTER(Params), P, P, P, P, P, I32, C.POINTER(Result)],
        "slk_fit": [P, I64, I32, P, I32, P, C.POINTER(Params), P, P, P, P, C.POINTER(Result)],
        "slk_energy": [P, I64, I32, P, I32, P, P, P, D, D, D, P, C.POINTER(EnergyOut)],
        "slk_unary": [P, I64, I32, I32, P, D, I32, P, P, P],
        "slk_inner_step": [P, I32, P, P, D, D, I32, P, P, P],
        "slk_inner_step_noalloc": [P, I32, P, P, D, D, I32, P, P, P],
        "slk_predict": [P, I64, I32, P, I32, P, P, I64, I32, D, D, I32, I32, P, P, P, P],
        "slk_mean_shift": [P, I64, I32, P, I32, P, D, D, I32, I32, P, P, P],
        "slk_fit_ms": [P, I64, I32, P, I32, P, C.POINTER(Params), D, I32, P, P, P, P, P, P, C.POINTER(Result)],
        "slk_kmeanspp": [P, I64, I32, I32, P, I32, P, P, P, P],
        "slk_dense_modes": [P, I64, I32, I32, P, P, D, P, P, I32, P, P, P, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.slk_inner_step_noalloc_max_rows.argtypes = [I32]
    lib.slk_inner_step_noalloc_max_rows.restype = I64
    lib.slk_pool_trim.argtypes = []
    lib.slk_pool_trim.restype = C.c_int
    lib.slk_timing_enable.argtypes = [I32]
    lib.slk_timing_enable.restype = C.c_int
    lib.slk_timing_read.argtypes = [C.c_char_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    lib.slk_timing_read.restype = C.c_int
    lib.slk_graph_destroy.argtypes = [P]
    lib.slk_graph_destroy.restype = None
    lib.slk_last_error.restype = C.c_char_p
    lib.slk_version.restype = C.c_char_p
    lib.slk_tune_source.restype = C.c_char_p
    srv = {
        "slk_server_opts_default": [C.POINTER(ServerOpts)],
        "slk_server_create": [C.POINTER(ServerOpts), P, C.POINTER(P)],
        "slk_server_submit": [P, C.POINTER(Job), C.POINTER(C.c_int64)],
        "slk_server_step": [P, P, I32, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32)],
        "slk_fit_batched": [C.POINTER(Job), I32, C.POINTER(ServerOpts), P],
        "slk_server_stats": [P, C.POINTER(ServerStats)],
        "slk_build_knn_batched": [C.POINTER(KnnItem), I32, P, C.POINTER(P)],
        "slk_tune_lookup": [I64, I32, I32, C.POINTER(TuneParams)],
        "slk_tune_override": [I32],
    }
    for name, args in srv.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.slk_server_destroy.argtypes = [P]
    lib.slk_server_destroy.restype = None
    _lib = lib
    return lib


def check(status: int):
    if status != SLK_OK:
        msg = load().slk_last_error().decode(errors="replace")
        raise SlkError(status, msg)


def host_i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def ptr_i32(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)
