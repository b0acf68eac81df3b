"""ctypes binding of the C ABI in ``include/cp_arls_lev.h``.

Argument marshalling only: every step of a mode update runs in the HIP
library ``libcpal.so``.  PyTorch provides device memory and the stream.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcpal.so")

CPAL_OK, CPAL_E_ARG, CPAL_E_NOMEM, CPAL_E_DEVICE, CPAL_E_STATE = 0, 1, 2, 3, 4
CPAL_F64, CPAL_F32, CPAL_BF16 = 0, 1, 2
SAMPLING = {"leverage": 0, "uniform": 1, "length_squared": 2}
FLAG_PINV, FLAG_DETCAP, FLAG_DET_TRUNC, FLAG_PDET_ONE, FLAG_DRAWCAP, FLAG_OVERFLOW, FLAG_STATE = (
    1, 2, 4, 8, 16, 32, 64)

# every extern "C" symbol declared in include/cp_arls_lev.h
SYMBOLS = (
    "cp_arls_lev_init", "cp_arls_lev_mode_update", "cp_arls_lev_fit_estimate",
    "cp_arls_lev_samples", "cp_arls_lev_leverage", "cp_arls_lev_refresh",
    "cp_arls_lev_leverage_noalloc", "cp_arls_lev_rrf_init",
    "cp_arls_lev_get_step", "cp_arls_lev_set_step", "cp_arls_lev_set_timing",
    "cp_arls_lev_stage_times", "cp_arls_lev_last_error", "cp_arls_lev_destroy",
    "cp_arls_lev_init_batch", "cp_arls_lev_mode_step_batch", "cp_arls_lev_fit_estimate_batch",
    "cp_arls_lev_batch_set_graphs", "cp_arls_lev_batch_graph_kernels", "cp_arls_lev_batch_ctx",
    "cp_arls_lev_destroy_batch",
    "cp_arls_lev_set_gather_config", "cp_arls_lev_get_gather_config", "cp_arls_lev_autotune",
    "cp_arls_lev_autotune_batch", "cp_arls_lev_fit_exact", "cp_arls_lev_run",
)
STAGES = ("sample", "rows", "gather", "solve", "leverage")


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class cpal_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", C.c_void_p)]


class cpal_tensor(C.Structure):
    _fields_ = [("order", C.c_int32), ("dims", C.POINTER(C.c_int64)), ("nnz", C.c_int64),
                ("coords", C.c_void_p), ("values", C.c_void_p), ("value_dtype", C.c_int32),
                ("dense", C.c_int32)]


class cpal_options(C.Structure):
    _fields_ = [("rank", C.c_int32), ("samples", C.c_int64), ("tau", C.c_double),
                ("seed", C.c_uint64), ("stream_id", C.c_uint64), ("gather_dtype", C.c_int32),
                ("fit_samples", C.c_int64), ("fit_nnz_fraction", C.c_double),
                ("det_enum_cap", C.c_int64), ("sampling", C.c_int32), ("pad", C.c_int32)]


class cpal_mode_stats(C.Structure):
    _fields_ = [("s_det", C.c_int64), ("s_rnd", C.c_int64), ("s_bar", C.c_int64),
                ("draws", C.c_int64), ("gathered_nnz", C.c_int64), ("p_det", C.c_double),
                ("flags", C.c_int32), ("pad", C.c_int32)]


class cpal_run_options(C.Structure):
    _fields_ = [("eta", C.c_int32), ("pi", C.c_int32), ("tol", C.c_double),
                ("max_epochs", C.c_int32), ("exact_fit", C.c_int32)]


class cpal_run_result(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("stopped", C.c_int32), ("best_fit", C.c_double),
                ("final_exact_fit", C.c_double)]


STATS_BYTES = C.sizeof(cpal_mode_stats)
_lib = None


def load(path: str | None = None):
    """Load libcpal.so and declare the C signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = LIB_PATH if path is None else path
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
    L = C.CDLL(path)
    P = C.POINTER
    vp = C.c_void_p
    L.cp_arls_lev_init.argtypes = [P(cpal_tensor), P(cpal_options), P(vp), vp,
                                   P(cpal_allocator), P(vp)]
    L.cp_arls_lev_init.restype = C.c_int
    L.cp_arls_lev_mode_update.argtypes = [vp, C.c_int32, vp]
    L.cp_arls_lev_mode_update.restype = C.c_int
    L.cp_arls_lev_fit_estimate.argtypes = [vp, vp]
    L.cp_arls_lev_fit_estimate.restype = C.c_int
    L.cp_arls_lev_fit_exact.argtypes = [vp, vp]
    L.cp_arls_lev_fit_exact.restype = C.c_int
    L.cp_arls_lev_run.argtypes = [vp, P(cpal_run_options), P(C.c_double), P(cpal_run_result)]
    L.cp_arls_lev_run.restype = C.c_int
    L.cp_arls_lev_samples.argtypes = [vp, vp, vp, vp, C.c_int64, vp]
    L.cp_arls_lev_samples.restype = C.c_int
    L.cp_arls_lev_leverage.argtypes = [vp, C.c_int32, vp]
    L.cp_arls_lev_leverage.restype = C.c_int
    L.cp_arls_lev_rrf_init.argtypes = [vp, C.c_int64, C.POINTER(vp)]
    L.cp_arls_lev_rrf_init.restype = C.c_int
    L.cp_arls_lev_leverage_noalloc.argtypes = [vp, C.c_int64, C.c_int32, vp, vp]
    L.cp_arls_lev_leverage_noalloc.restype = C.c_int
    L.cp_arls_lev_refresh.argtypes = [vp, C.c_int32]
    L.cp_arls_lev_refresh.restype = C.c_int
    L.cp_arls_lev_get_step.argtypes = [vp, P(C.c_uint64)]
    L.cp_arls_lev_get_step.restype = C.c_int
    L.cp_arls_lev_set_step.argtypes = [vp, C.c_uint64]
    L.cp_arls_lev_set_step.restype = C.c_int
    L.cp_arls_lev_set_timing.argtypes = [vp, C.c_int32]
    L.cp_arls_lev_set_timing.restype = C.c_int
    L.cp_arls_lev_stage_times.argtypes = [vp, P(C.c_double), P(C.c_int64), C.c_int32]
    L.cp_arls_lev_stage_times.restype = C.c_int
    L.cp_arls_lev_last_error.argtypes = [vp]
    L.cp_arls_lev_last_error.restype = C.c_char_p
    L.cp_arls_lev_destroy.argtypes = [vp]
    L.cp_arls_lev_destroy.restype = None
    L.cp_arls_lev_init_batch.argtypes = [C.c_int32, P(cpal_tensor), C.c_int32, P(C.c_int32),
                                         P(cpal_options), P(vp), vp, P(cpal_allocator),
                                         P(vp)]
    L.cp_arls_lev_init_batch.restype = C.c_int
    L.cp_arls_lev_mode_step_batch.argtypes = [vp, C.c_int32, vp]
    L.cp_arls_lev_mode_step_batch.restype = C.c_int
    L.cp_arls_lev_fit_estimate_batch.argtypes = [vp, vp]
    L.cp_arls_lev_fit_estimate_batch.restype = C.c_int
    L.cp_arls_lev_set_gather_config.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
    L.cp_arls_lev_set_gather_config.restype = C.c_int
    L.cp_arls_lev_get_gather_config.argtypes = [vp, C.c_int32, P(C.c_int32), P(C.c_int32)]
    L.cp_arls_lev_get_gather_config.restype = C.c_int
    L.cp_arls_lev_autotune.argtypes = [vp, C.c_int32]
    L.cp_arls_lev_autotune.restype = C.c_int
    L.cp_arls_lev_autotune_batch.argtypes = [vp, C.c_int32]
    L.cp_arls_lev_autotune_batch.restype = C.c_int
    L.cp_arls_lev_batch_set_graphs.argtypes = [vp, C.c_int32]
    L.cp_arls_lev_batch_set_graphs.restype = C.c_int
    L.cp_arls_lev_batch_graph_kernels.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]
    L.cp_arls_lev_batch_graph_kernels.restype = C.c_int
    L.cp_arls_lev_batch_ctx.argtypes = [vp, C.c_int32, P(vp)]
    L.cp_arls_lev_batch_ctx.restype = C.c_int
    L.cp_arls_lev_destroy_batch.argtypes = [vp]
    L.cp_arls_lev_destroy_batch.restype = None
    _lib = L
    return L


class CpalError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"cp_arls_lev error {code}: {msg}")
        self.code = code
