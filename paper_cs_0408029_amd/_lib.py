"""ctypes binding of the C ABI declared in include/nnls.h.

Only argument marshalling lives here: every step of the solver runs in the HIP kernels of
lib/libnnls.so.  Loading fails loudly when the library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libnnls.so")

NNLS_OK = 0
NNLS_ERR_INVALID_ARG = -1
NNLS_ERR_INVALID_VALUE = -2
NNLS_ERR_NOT_PD = -3
NNLS_ERR_MAXITER = -4
NNLS_ERR_NO_MEMORY = -5
NNLS_ERR_DEVICE = -6
NNLS_ERR_REFINE = -7
NNLS_ERR_TIMEOUT = -8
NNLS_ERR_TOO_LARGE = -9

# bytes of the fixed device array behind nnls_solve_dense_batched_noalloc
NNLS_NOALLOC_SCRATCH_BYTES = 64 << 20

NNLS_FP64 = 0
NNLS_FP32_IR = 1
NNLS_BF16_IR = 2

NNLS_FLAG_PROFILE = 1
NNLS_FLAG_REFINE_FINAL = 2
NNLS_FLAG_NO_FACTOR_REUSE = 4
NNLS_FLAG_REFINE_AUTO = 8
NNLS_FLAG_GRAM_DUAL = 16
NNLS_FLAG_REFINE_ALL = 32

NNLS_PROFILE_CLASSES = 9
PROFILE_CLASS_NAMES = ["gram", "control", "cholesky", "trsv", "residual", "refine", "batched", "dual",
                       "batched_gram"]


class nnls_options(C.Structure):
    _fields_ = [("tau", C.c_double), ("p_max", C.c_int32), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("ir_max_steps", C.c_int32), ("ir_rtol", C.c_double),
                ("flags", C.c_uint32), ("max_workgroups", C.c_uint32)]


class nnls_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("n_free", C.c_int32),
                ("last_ninf", C.c_int32), ("failed_index", C.c_int32), ("ir_steps", C.c_int32),
                ("min_margin", C.c_double), ("setup_ms", C.c_double), ("solve_ms", C.c_double),
                ("est_rel_err", C.c_double)]


class nnls_trace_row(C.Structure):
    _fields_ = [("k", C.c_int32), ("branch", C.c_int32), ("N", C.c_int32), ("p", C.c_int32),
                ("n_free", C.c_int32), ("n_reused", C.c_int32), ("ir_steps", C.c_int32)]


class nnls_server_config(C.Structure):
    _fields_ = [("hbm_budget", C.c_size_t), ("workers", C.c_int32), ("batch_lanes", C.c_int32),
                ("batch_max_n", C.c_int32), ("batch_max_count", C.c_int32), ("batch_step_iters", C.c_int32),
                ("pad", C.c_int32)]


class nnls_serving_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("pending", C.c_int64),
                ("batches", C.c_int64), ("running", C.c_int32), ("max_running", C.c_int32),
                ("committed_bytes", C.c_double), ("peak_committed_bytes", C.c_double),
                ("budget_bytes", C.c_double), ("p50_ms", C.c_double), ("p99_ms", C.c_double),
                ("mean_ms", C.c_double), ("max_ms", C.c_double), ("solves_per_s", C.c_double)]


_P = C.c_void_p
_I32 = C.c_int32
_I64 = C.c_int64

# name -> (restype, argtypes), in the order of include/nnls.h
PROTOTYPES = {
    "nnls_status_string": (C.c_char_p, [C.c_int]),
    "nnls_default_options": (None, [C.POINTER(nnls_options)]),
    "nnls_create": (C.c_int, [C.POINTER(_P), C.c_int, _P]),
    "nnls_destroy": (C.c_int, [_P]),
    "nnls_solve_csc": (C.c_int, [_P, _I32, _I32, _I64, _P, _P, _P, _P, _P, _P,
                                 C.POINTER(nnls_options), C.POINTER(nnls_info)]),
    "nnls_solve_dense": (C.c_int, [_P, _I32, _I32, _P, _I32, _P, _P, _P,
                                   C.POINTER(nnls_options), C.POINTER(nnls_info)]),
    "nnls_solve_dense_batched": (C.c_int, [_P, _I32, _P, _P, _P, _P, _P, _P, _P,
                                           C.POINTER(nnls_options), _P]),
    "nnls_solve_dense_batched_noalloc": (C.c_int, [_P, _I32, _P, _P, _P, _P, _P, _P, _P,
                                                   C.POINTER(nnls_options), _P]),
    "nnls_batch_plan_create": (C.c_int, [_P, _I32, _P, _P, _P, _P, _P, _P, _P, C.POINTER(nnls_options),
                                         C.POINTER(_P)]),
    "nnls_batch_plan_execute": (C.c_int, [_P, _P]),
    "nnls_batch_plan_info": (C.c_int, [_P, _P]),
    "nnls_batch_plan_destroy": (C.c_int, [_P]),
    "nnls_batch_plan_tile_shapes": (C.c_int, [_P, _P]),
    "nnls_server_create": (C.c_int, [C.POINTER(_P), C.c_int, C.POINTER(nnls_server_config),
                                     C.POINTER(nnls_options)]),
    "nnls_server_submit_csc": (C.c_int, [_P, _I32, _I32, _I64, _P, _P, _P, _P, C.POINTER(C.c_uint64)]),
    "nnls_server_poll": (C.c_int, [_P, C.c_uint64, C.POINTER(_I32), _P, _P, C.POINTER(nnls_info)]),
    "nnls_server_wait": (C.c_int, [_P, C.c_uint64, C.c_double, _P, _P, C.POINTER(nnls_info)]),
    "nnls_server_stats": (C.c_int, [_P, C.POINTER(nnls_serving_stats)]),
    "nnls_server_reset_stats": (C.c_int, [_P]),
    "nnls_server_destroy": (C.c_int, [_P]),
    "nnls_get_trace": (C.c_int, [_P, C.POINTER(nnls_trace_row), C.c_int]),
    "nnls_get_profile": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]),
    "nnls_reset_profile": (C.c_int, [_P]),
    "nnls_set_profiling": (C.c_int, [_P, C.c_int]),
    "nnls_gram_csc": (C.c_int, [_P, _I32, _I32, _I64, _P, _P, _P, _P, _P, _I32, _P]),
    "nnls_gram_dense": (C.c_int, [_P, _I32, _I32, _P, _I32, _P, _P, _I32, _P]),
    "nnls_cholesky": (C.c_int, [_P, _I32, _P, _I32, _P, _I32, _I32, C.POINTER(_I32)]),
    "nnls_spd_solve": (C.c_int, [_P, _I32, _P, _I32, _P, _P, C.POINTER(_I32)]),
    "nnls_dual_csc": (C.c_int, [_P, _I32, _I32, _I64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "nnls_dual_dense": (C.c_int, [_P, _I32, _I32, _P, _I32, _P, _P, _P, _P, _P]),
    "nnls_pivot_step": (C.c_int, [_P, _I32, _P, _P, _P, C.c_double, _I32, C.POINTER(_I32),
                                  C.POINTER(_I32)]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load lib/libnnls.so and attach the prototypes.  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"native library not built: {path} (run __graft_entry__.build())")
    lib = C.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(st: int) -> str:
    return load().nnls_status_string(st).decode()


def default_options(**overrides) -> nnls_options:
    o = nnls_options()
    load().nnls_default_options(C.byref(o))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o
