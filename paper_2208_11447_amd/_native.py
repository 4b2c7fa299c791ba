"""ctypes declarations of the libskfab C ABI (include/skfab.h).

Argument marshalling only: every numerical step runs in the HIP library.  The
library must be built (``paper_2208_11447_amd.build_lib.build()``); loading
fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libskfab.so")

SKFAB_OK, SKFAB_ERR_ARG, SKFAB_ERR_SHAPE, SKFAB_ERR_RANK, SKFAB_ERR_BRANCH, SKFAB_ERR_QUAD, \
    SKFAB_ERR_HIP, SKFAB_ERR_WORKSPACE, SKFAB_ERR_TOO_LARGE = range(9)
SKFAB_NOALLOC_WS_BYTES = 64 * 1024 * 1024
SKFAB_F_INVSQRT, SKFAB_F_EXP, SKFAB_F_INV, SKFAB_F_POLY = range(4)
SKFAB_SFOM_CLOSED, SKFAB_SFOM_QUAD, SKFAB_SGMRES_QUAD = range(3)
SKFAB_PREC_FP64, SKFAB_PREC_FP32, SKFAB_PREC_FP32_BF16BASIS = range(3)
SKFAB_VAL_F64 = 0
SKFAB_FLAG_TRUNCATED, SKFAB_FLAG_QUAD_FLOOR = 1, 2
SKFAB_SKETCH_SPARSE_SIGN, SKFAB_SKETCH_SRDCT = 0, 1

EXPORTED = [
    "skfab_version", "skfab_status_string", "skfab_create", "skfab_set_stream", "skfab_destroy",
    "skfab_workspace_bytes", "skfab_solve", "skfab_solve_noalloc", "skfab_solve_reckless", "skfab_arnoldi",
    "skfab_small_problem",
    "skfab_small_workspace_bytes", "skfab_sketch_pattern", "skfab_sketch_apply", "skfab_sketch_ws_bytes",
    "skfab_timing_enable", "skfab_timing_read", "skfab_set_value_table", "skfab_set_arnoldi_check", "skfab_srdct_ws_bytes",
    "skfab_srdct_apply",
    "skfab_batch_workspace_bytes", "skfab_solve_batched", "skfab_batch_set_tuning", "skfab_batch_get_tuning",
    "skfab_batch_autotune",
    "skfab_adaptive_workspace_bytes", "skfab_solve_adaptive", "skfab_gershgorin_ws_bytes", "skfab_gershgorin",
    "skfab_mlp_param_count", "skfab_mlp_ws_bytes", "skfab_mlp_forward", "skfab_mlp_loss_grad", "skfab_mlp_adam",
]


class skfab_csr(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p), ("val_type", C.c_int32)]


class skfab_params(C.Structure):
    _fields_ = [("f", C.c_int32), ("fparam", C.c_double), ("poly", C.POINTER(C.c_double)),
                ("npoly", C.c_int32), ("method", C.c_int32), ("m", C.c_int32), ("k", C.c_int32),
                ("s", C.c_int32), ("zeta", C.c_int32), ("seed", C.c_uint64), ("l1", C.c_int32),
                ("l2", C.c_int32), ("lmax", C.c_int32), ("quad_tol", C.c_double), ("prec", C.c_int32),
                ("cond_max", C.c_double), ("sketch", C.c_int32), ("srdct_signs", C.c_void_p),
                ("srdct_rows", C.c_void_p), ("two_pass", C.c_int32)]


class skfab_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("m_used", C.c_int32), ("l_used", C.c_int32),
                ("a_format", C.c_int32), ("eps_est", C.c_double), ("rcond_R", C.c_double),
                ("sigma", C.c_double), ("beta", C.c_double), ("arnoldi_relres", C.c_double),
                ("quad_diff", C.c_double), ("flags", C.c_int32), ("m_basis", C.c_int32)]


class skfab_batch_problem(C.Structure):
    _fields_ = [("A", skfab_csr), ("B", C.c_void_p), ("X", C.c_void_p), ("m", C.c_int32), ("s", C.c_int32),
                ("seed", C.c_uint64), ("ldb", C.c_int64), ("ldx", C.c_int64)]


class skfab_batch_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("slices_per_wave", C.c_int32), ("packed", C.c_int32)]


_lib = None


def lib():
    """Load libskfab.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -m paper_2208_11447_amd.build_lib)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "skfab_version": (C.c_int32, []),
        "skfab_status_string": (C.c_char_p, [C.c_int32]),
        "skfab_create": (C.c_int, [C.POINTER(P), C.c_int32, P]),
        "skfab_set_stream": (C.c_int, [P, P]),
        "skfab_destroy": (C.c_int, [P]),
        "skfab_workspace_bytes": (C.c_int, [C.POINTER(skfab_csr), C.POINTER(skfab_params), C.c_int32,
                                             C.POINTER(C.c_size_t)]),
        "skfab_solve": (C.c_int, [P, C.POINTER(skfab_csr), P, C.c_int64, C.c_int32, P, C.c_int64,
                                  C.POINTER(skfab_params), P, C.c_size_t, C.POINTER(skfab_info)]),
        "skfab_solve_noalloc": (C.c_int, [P, C.POINTER(skfab_csr), P, P, C.POINTER(skfab_params),
                                          C.POINTER(skfab_info)]),
        "skfab_solve_reckless": (C.c_int, [P, C.POINTER(skfab_csr), P, P, C.POINTER(skfab_params), C.c_int32,
                                           C.c_double, P, C.c_size_t, C.POINTER(skfab_info),
                                           C.POINTER(C.c_int32)]),
        "skfab_arnoldi": (C.c_int, [P, C.POINTER(skfab_csr), P, C.POINTER(skfab_params), P, P, P, P, P,
                                    C.c_size_t, C.POINTER(skfab_info)]),
        "skfab_small_problem": (C.c_int, [P, P, P, C.c_double, C.POINTER(skfab_params), P, P, C.c_size_t,
                                          C.POINTER(skfab_info)]),
        "skfab_small_workspace_bytes": (C.c_int, [C.POINTER(skfab_params), C.POINTER(C.c_size_t)]),
        "skfab_sketch_pattern": (C.c_int, [P, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_uint64, P, P]),
        "skfab_sketch_apply": (C.c_int, [P, C.c_int64, C.c_int32, C.c_int32, C.c_uint64, P, P, P, C.c_size_t]),
        "skfab_sketch_ws_bytes": (C.c_size_t, [C.c_int64, C.c_int32]),
        "skfab_timing_enable": (C.c_int, [P, C.c_int32]),
        "skfab_srdct_ws_bytes": (C.c_size_t, [C.c_int64, C.c_int32, C.c_int32]),
        "skfab_srdct_apply": (C.c_int, [P, C.c_int64, C.c_int32, P, P, P, C.c_int64, C.c_int32, P, P, C.c_size_t]),
        "skfab_set_value_table": (C.c_int, [P, C.c_int32]),
        "skfab_set_arnoldi_check": (C.c_int, [P, C.c_int32]),
        "skfab_timing_read": (C.c_int, [P, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "skfab_batch_workspace_bytes": (C.c_int, [C.c_int32, C.POINTER(skfab_batch_problem), C.c_int32,
                                                  C.POINTER(skfab_params), C.POINTER(C.c_size_t)]),
        "skfab_solve_batched": (C.c_int, [P, C.c_int32, C.POINTER(skfab_batch_problem), C.c_int32,
                                          C.POINTER(skfab_params), P, C.c_size_t, C.POINTER(skfab_info)]),
        "skfab_batch_set_tuning": (C.c_int, [P, C.POINTER(skfab_batch_tuning)]),
        "skfab_batch_get_tuning": (C.c_int, [P, C.POINTER(skfab_batch_tuning)]),
        "skfab_batch_autotune": (C.c_int, [P, C.c_int32, C.POINTER(skfab_batch_problem), C.c_int32,
                                           C.POINTER(skfab_params), P, C.c_size_t, C.c_int32,
                                           C.POINTER(skfab_batch_tuning)]),
        "skfab_adaptive_workspace_bytes": (C.c_int, [C.POINTER(skfab_csr), C.POINTER(skfab_params),
                                                     C.POINTER(C.c_size_t)]),
        "skfab_solve_adaptive": (C.c_int, [P, C.POINTER(skfab_csr), P, P, C.POINTER(skfab_params), C.c_int32,
                                           C.c_int32, C.c_double, P, C.c_size_t, C.POINTER(skfab_info),
                                           C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
        "skfab_gershgorin_ws_bytes": (C.c_size_t, [C.c_int64]),
        "skfab_gershgorin": (C.c_int, [P, C.POINTER(skfab_csr), P, P, C.c_size_t]),
        "skfab_mlp_param_count": (C.c_int32, []),
        "skfab_mlp_ws_bytes": (C.c_size_t, [C.c_int32]),
        "skfab_mlp_forward": (C.c_int, [P, P, C.c_int32, P, P, P, C.c_size_t]),
        "skfab_mlp_loss_grad": (C.c_int, [P, P, P, C.c_int32, P, P, P, P, C.c_size_t]),
        "skfab_mlp_adam": (C.c_int, [P, P, P, P, P, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L
