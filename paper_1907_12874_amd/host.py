"""Python front end of the host executor (libbicgstab_host.so, C ABI in
include/bicgstab_host.h): the GPU library's launch plans run on the host's
cores with OpenMP, for the merged-versus-basic comparison the paper made on
CPU nodes (Section 3.1.3, Table 4) and as a multi-core CPU baseline.

This is a separate solver with its own entry points; the GPU solver never
calls it. Argument marshalling only: numpy arrays in host memory.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from ._lib import FORMULATIONS, PRECONDS, VARIANTS, BicgstabError, Info

LIB_HOST_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbicgstab_host.so")

_libh = None


class HostCSRDesc(C.Structure):
    _fields_ = [
        ("n", C.c_int64),
        ("nnz", C.c_int64),
        ("row_ptr", C.c_void_p),
        ("col_idx", C.c_void_p),
        ("values", C.c_void_p),
    ]


def lib_host():
    """Load the built host executor (raises if it has not been built)."""
    global _libh
    if _libh is not None:
        return _libh
    if not os.path.exists(LIB_HOST_PATH):
        raise RuntimeError(f"{LIB_HOST_PATH} is missing: build it with `python -m paper_1907_12874_amd.build`")
    L = C.CDLL(LIB_HOST_PATH)
    H, i32, dbl, vp = C.c_void_p, C.c_int32, C.c_double, C.c_void_p
    L.bicgstab_host_create.argtypes = [C.POINTER(HostCSRDesc), i32, i32, i32, i32, i32, C.POINTER(H)]
    L.bicgstab_host_solve.argtypes = [H, vp, vp, dbl, i32, C.POINTER(Info)]
    L.bicgstab_host_loop_time.argtypes = [H, C.POINTER(dbl), C.POINTER(i32)]
    L.bicgstab_host_destroy.argtypes = [H]
    L.bicgstab_host_axpby_tab1.argtypes = [i32, C.c_int64, dbl, dbl, dbl, vp, vp, vp, i32]
    L.bicgstab_host_last_error.argtypes = []
    L.bicgstab_host_last_error.restype = C.c_char_p
    _libh = L
    return L


def _check(code, where):
    if code != 0:
        raise BicgstabError(code, where, lib_host().bicgstab_host_last_error().decode())


def axpby_tab1(run: int, x, y, z, a: float, b: float, c: float, threads: int = 1):
    """Table 1's vector updates on host float64 arrays (y and z updated in
    place): run 1 as three passes, run 2 the first two merged, run 3 all
    three merged."""
    for t, name in ((x, "x"), (y, "y"), (z, "z")):
        if not (isinstance(t, np.ndarray) and t.dtype == np.float64 and t.flags.c_contiguous and t.size == x.size):
            raise ValueError(f"{name} must be a contiguous float64 array of length {x.size}")
    _check(lib_host().bicgstab_host_axpby_tab1(int(run), int(x.size), float(a), float(b), float(c), x.ctypes.data,
                                               y.ctypes.data, z.ctypes.data, int(threads)), "bicgstab_host_axpby_tab1")


class HostSolver:
    """The same methods as Solver on the host's cores: A in CSR (numpy
    int32 / float64 arrays, copied), k right-hand sides, `threads` fixed row
    ranges per pass (dot products summed per range, then over ranges, in
    order: bitwise repeatable for a given thread count)."""

    def __init__(self, row_ptr, col_idx, values, k: int, variant: str = "classical", formulation: str = "merged",
                 precond: str = "none", threads: int = 1):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        va = np.ascontiguousarray(values, dtype=np.float64)
        self.n, self.k, self.threads = int(rp.size) - 1, int(k), int(threads)
        self.variant, self.formulation, self.precond = variant, formulation, precond
        desc = HostCSRDesc(self.n, int(ci.size), rp.ctypes.data, ci.ctypes.data, va.ctypes.data)
        h = C.c_void_p()
        _check(lib_host().bicgstab_host_create(C.byref(desc), self.k, VARIANTS[variant], FORMULATIONS[formulation],
                                               PRECONDS[precond], self.threads, C.byref(h)),
               "bicgstab_host_create")
        self._h = h

    @classmethod
    def from_csr(cls, A, k: int, **kw):
        return cls(A.row_ptr, A.col_idx, A.values, k, **kw)

    def solve(self, b, x0=None, tol: float = 1e-8, maxit: int = 1000):
        """Solve A X = B; returns (X, SolveInfo) with X a new n x k array."""
        from .solver import SolveInfo

        b = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(self.n, self.k))
        x = np.zeros((self.n, self.k)) if x0 is None else np.array(x0, dtype=np.float64).reshape(self.n, self.k)
        x = np.ascontiguousarray(x)
        arrs = (np.zeros(self.k, np.int32), np.zeros(self.k, np.int32), np.zeros(self.k), np.zeros(self.k))
        info = Info(arrs[0].ctypes.data_as(C.POINTER(C.c_int32)), arrs[1].ctypes.data_as(C.POINTER(C.c_int32)),
                    arrs[2].ctypes.data_as(C.POINTER(C.c_double)), arrs[3].ctypes.data_as(C.POINTER(C.c_double)))
        _check(lib_host().bicgstab_host_solve(self._h, b.ctypes.data, x.ctypes.data, float(tol), int(maxit),
                                              C.byref(info)), "bicgstab_host_solve")
        return x, SolveInfo(*arrs)

    def loop_time(self):
        """(seconds, passes) of the last solve's iteration loop."""
        sec, passes = C.c_double(), C.c_int32()
        _check(lib_host().bicgstab_host_loop_time(self._h, C.byref(sec), C.byref(passes)), "bicgstab_host_loop_time")
        return sec.value, passes.value

    def close(self):
        if getattr(self, "_h", None):
            lib_host().bicgstab_host_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
