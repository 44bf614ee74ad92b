"""ctypes declarations of the C ABI in include/bicgstab.h."""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbicgstab.so")

OK, EINVAL, EHIP, ENOMEM, EUNSUPPORTED = 0, -1, -2, -3, -4
VARIANTS = {"classical": 0, "reordered": 1, "pipelined": 2, "improved": 3}
FORMULATIONS = {"merged": 0, "basic": 1, "fused": 2}
PRECONDS = {"none": 0, "jacobi": 1}
PRECISIONS = {"fp64": 0, "fp32_refine": 1}
STATUS_NAMES = {0: "converged", 1: "maxit", 2: "breakdown", 3: "nonfinite"}
MAX_K = 64


class CSRDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("nnz", C.c_int64),
        ("d_row_ptr", C.c_void_p),
        ("d_col_idx", C.c_void_p),
        ("d_values", C.c_void_p),
    ]


class Info(C.Structure):
    _fields_ = [
        ("iters", C.POINTER(C.c_int32)),
        ("status", C.POINTER(C.c_int32)),
        ("relres_true", C.POINTER(C.c_double)),
        ("relres_recursive", C.POINTER(C.c_double)),
    ]


_lib = None


class BicgstabError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


def lib():
    """Load the built HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1907_12874_amd.build` "
            "(the solver has no fallback path)"
        )
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    H = C.c_void_p
    L.bicgstab_create.argtypes = [C.POINTER(CSRDesc), i64, i32, i32, i32, i32, i32, vp, C.POINTER(H)]
    L.bicgstab_workspace_bytes.argtypes = [H, C.POINTER(C.c_size_t)]
    L.bicgstab_set_workspace.argtypes = [H, vp, C.c_size_t]
    L.bicgstab_set_stream.argtypes = [H, vp]
    L.bicgstab_solve.argtypes = [H, vp, vp, dbl, i32, C.POINTER(Info)]
    L.bicgstab_solve_noalloc.argtypes = [H, vp, vp, dbl, i32, C.POINTER(Info)]
    L.bicgstab_solve_transpose.argtypes = [H, vp, vp, dbl, i32, C.POINTER(Info)]
    L.bicgstab_grad_values.argtypes = [H, vp, vp, vp]
    L.bicgstab_update_values.argtypes = [H, C.c_void_p]
    L.bicgstab_spmm.argtypes = [H, vp, vp]
    L.bicgstab_product_layout.argtypes = [H, C.POINTER(i32), C.POINTER(i32)]
    L.bicgstab_history.argtypes = [H, C.POINTER(dbl), i32, C.POINTER(i32)]
    L.bicgstab_last_solve_stats.argtypes = [H, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    L.bicgstab_refine_outer.argtypes = [H, C.POINTER(i32)]
    L.bicgstab_destroy.argtypes = [H]
    L.bicgstab_plan_traffic.argtypes = [i32, i32, i32] + [C.POINTER(i32)] * 5
    L.bicgstab_axpby_tab1.argtypes = [i32, i64, dbl, dbl, dbl, vp, vp, vp, vp]
    L.bicgstab_strerror.argtypes = [C.c_int]
    L.bicgstab_strerror.restype = C.c_char_p
    L.bicgstab_last_error.argtypes = []
    L.bicgstab_last_error.restype = C.c_char_p
    L.bicgstab_kernel_times.argtypes = [H, vp, vp, i32, i32] + [C.POINTER(i32)] * 4 + [C.POINTER(dbl), C.POINTER(i32)]
    L.bicgstab_batched_create.argtypes = [C.POINTER(CSRDesc), C.POINTER(i32), i32, i32, i32, vp, C.POINTER(H)]
    L.bicgstab_batched_workspace_bytes.argtypes = [H, C.POINTER(C.c_size_t)]
    L.bicgstab_batched_set_workspace.argtypes = [H, vp, C.c_size_t]
    L.bicgstab_batched_set_stream.argtypes = [H, vp]
    L.bicgstab_batched_solve.argtypes = [H, C.POINTER(vp), C.POINTER(vp), dbl, i32, C.POINTER(Info)]
    L.bicgstab_batched_tune.argtypes = [H, C.POINTER(vp), C.POINTER(vp), dbl, i32, C.POINTER(dbl)]
    L.bicgstab_batched_get_config.argtypes = [H, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), C.POINTER(dbl),
                                              C.POINTER(dbl)]
    L.bicgstab_batched_variant_info.argtypes = [i32] + [C.POINTER(i32)] * 4
    L.bicgstab_batched_set_config.argtypes = [H, i32, C.POINTER(i32)]
    L.bicgstab_batched_destroy.argtypes = [H]
    _lib = L
    return L


def check(code: int, where: str):
    if code != OK:
        L = lib()
        raise BicgstabError(code, where, L.bicgstab_last_error().decode() or L.bicgstab_strerror(code).decode())


def exported_symbols():
    """Names the ABI header declares (for the symbol-export test)."""
    return [
        "bicgstab_create", "bicgstab_workspace_bytes", "bicgstab_set_workspace", "bicgstab_set_stream",
        "bicgstab_solve", "bicgstab_solve_transpose", "bicgstab_grad_values", "bicgstab_update_values",
        "bicgstab_spmm", "bicgstab_history", "bicgstab_last_solve_stats", "bicgstab_destroy",
        "bicgstab_plan_traffic", "bicgstab_strerror", "bicgstab_last_error", "bicgstab_kernel_times",
        "bicgstab_refine_outer", "bicgstab_batched_create", "bicgstab_batched_workspace_bytes",
        "bicgstab_batched_set_workspace", "bicgstab_batched_set_stream", "bicgstab_batched_solve",
        "bicgstab_batched_tune", "bicgstab_batched_get_config", "bicgstab_batched_set_config",
        "bicgstab_batched_variant_info", "bicgstab_batched_destroy", "bicgstab_axpby_tab1",
        "bicgstab_solve_noalloc", "bicgstab_product_layout",
    ]
