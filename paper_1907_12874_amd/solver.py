"""Python front end of the HIP library: argument marshalling only.

Every step of a solve runs in the library's kernels; PyTorch provides the
device memory (matrix arrays, right-hand sides, the workspace) and the stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check, lib


@dataclass
class SolveInfo:
    iters: np.ndarray
    status: np.ndarray
    relres_true: np.ndarray
    relres_recursive: np.ndarray

    @property
    def converged(self) -> bool:
        return bool(np.all(self.status == 0))


def _stream_ptr(device) -> int:
    return int(torch.cuda.current_stream(device).cuda_stream)


def _dev_tensor(t, dtype, device, name):
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t))
    t = t.to(device=device, dtype=dtype)
    if not t.is_contiguous():
        t = t.contiguous()
    return t


class Solver:
    """BiCGStab for A X = B with k right-hand sides on one GPU.

    A is given in CSR form (row_ptr int32 n+1, col_idx int32 nnz, values
    float64 nnz); the tensors are moved to the device once and kept alive for
    the life of the solver (the library borrows them).
    """

    def __init__(self, row_ptr, col_idx, values, k: int, variant: str = "classical", formulation: str = "merged",
                 precond: str = "none", precision: str = "fp64", device="cuda"):
        self.device = torch.device(device)
        self.row_ptr = _dev_tensor(row_ptr, torch.int32, self.device, "row_ptr")
        self.col_idx = _dev_tensor(col_idx, torch.int32, self.device, "col_idx")
        self.values = _dev_tensor(values, torch.float64, self.device, "values")
        self.n = int(self.row_ptr.numel()) - 1
        self.nnz = int(self.col_idx.numel())
        self.k = int(k)
        self.variant, self.formulation, self.precond, self.precision = variant, formulation, precond, precision
        # bumped by every update_values: lets a differentiable solve tell
        # whether the values it was run with are still the solver's
        self.values_version = 0
        L = lib()
        desc = _lib.CSRDesc(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(), self.values.data_ptr())
        self._desc = desc
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(L.bicgstab_create(C.byref(desc), self.n, self.k, _lib.VARIANTS[variant],
                                    _lib.FORMULATIONS[formulation], _lib.PRECONDS[precond],
                                    _lib.PRECISIONS[precision], C.c_void_p(_stream_ptr(self.device)), C.byref(h)),
                  "bicgstab_create")
        self._h = h
        nbytes = C.c_size_t()
        check(L.bicgstab_workspace_bytes(h, C.byref(nbytes)), "bicgstab_workspace_bytes")
        self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        check(L.bicgstab_set_workspace(h, C.c_void_p(self.workspace.data_ptr()), self.workspace.numel()),
              "bicgstab_set_workspace")

    @classmethod
    def from_csr(cls, A, k: int, **kw):
        """From a host CSR object with row_ptr / col_idx / values arrays."""
        return cls(torch.from_numpy(np.asarray(A.row_ptr, dtype=np.int32)),
                   torch.from_numpy(np.asarray(A.col_idx, dtype=np.int32)),
                   torch.from_numpy(np.asarray(A.values, dtype=np.float64)), k, **kw)

    # ---------------------------------------------------------------- helpers
    def _block(self, t, name):
        t = _dev_tensor(t, torch.float64, self.device, name)
        if t.dim() == 1 and self.k == 1:
            t = t.view(-1, 1)
        if tuple(t.shape) != (self.n, self.k):
            raise ValueError(f"{name} must be {self.n} x {self.k}, got {tuple(t.shape)}")
        return t

    def _set_stream(self):
        check(lib().bicgstab_set_stream(self._h, C.c_void_p(_stream_ptr(self.device))), "bicgstab_set_stream")

    def _info_struct(self):
        k = self.k
        arrs = (np.zeros(k, np.int32), np.zeros(k, np.int32), np.zeros(k, np.float64), np.zeros(k, np.float64))
        info = _lib.Info(arrs[0].ctypes.data_as(C.POINTER(C.c_int32)), arrs[1].ctypes.data_as(C.POINTER(C.c_int32)),
                         arrs[2].ctypes.data_as(C.POINTER(C.c_double)), arrs[3].ctypes.data_as(C.POINTER(C.c_double)))
        return info, arrs

    # -------------------------------------------------------------------- API
    def solve(self, b, x0=None, tol: float = 1e-8, maxit: int = 1000, out=None):
        """Solve A X = B. Returns (X, SolveInfo). x0 (optional) is copied."""
        b = self._block(b, "b")
        if out is not None:
            x = out
            if x0 is not None:
                x.copy_(self._block(x0, "x0"))
        else:
            x = torch.zeros_like(b) if x0 is None else self._block(x0, "x0").clone()
        info, arrs = self._info_struct()
        with torch.cuda.device(self.device):
            self._set_stream()
            check(lib().bicgstab_solve(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), float(tol),
                                       int(maxit), C.byref(info)), "bicgstab_solve")
        return x, SolveInfo(*arrs)

    def solve_noalloc(self, b, x0=None, tol: float = 1e-8, maxit: int = 1000, out=None):
        """solve() through bicgstab_solve_noalloc: the library's static device
        scratch is the workspace of the call (no device allocation in the
        library; the tensors here are the caller's). Returns (X, SolveInfo)."""
        b = self._block(b, "b")
        if out is not None:
            x = out
            if x0 is not None:
                x.copy_(self._block(x0, "x0"))
        else:
            x = torch.zeros_like(b) if x0 is None else self._block(x0, "x0").clone()
        info, arrs = self._info_struct()
        with torch.cuda.device(self.device):
            self._set_stream()
            check(lib().bicgstab_solve_noalloc(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                               float(tol), int(maxit), C.byref(info)), "bicgstab_solve_noalloc")
        return x, SolveInfo(*arrs)

    def solve_transpose(self, g, tol: float = 1e-8, maxit: int = 1000):
        """Solve A^T L = G from L = 0. Returns (L, SolveInfo)."""
        g = self._block(g, "g")
        lam = torch.zeros_like(g)
        info, arrs = self._info_struct()
        with torch.cuda.device(self.device):
            self._set_stream()
            check(lib().bicgstab_solve_transpose(self._h, C.c_void_p(g.data_ptr()), C.c_void_p(lam.data_ptr()),
                                                 float(tol), int(maxit), C.byref(info)), "bicgstab_solve_transpose")
        return lam, SolveInfo(*arrs)

    def grad_values(self, lam, x):
        """-sum_c lam[i, c] x[j, c] for every stored entry (i, j)."""
        lam = self._block(lam, "lam")
        x = self._block(x, "x")
        g = torch.empty(self.nnz, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            self._set_stream()
            check(lib().bicgstab_grad_values(self._h, C.c_void_p(lam.data_ptr()), C.c_void_p(x.data_ptr()),
                                             C.c_void_p(g.data_ptr())), "bicgstab_grad_values")
        return g

    def update_values(self, values):
        """Replace the matrix values (same pattern)."""
        v = _dev_tensor(values, torch.float64, self.device, "values")
        if v.numel() != self.nnz:
            raise ValueError("values must have nnz entries")
        self.values.copy_(v)
        with torch.cuda.device(self.device):
            self._set_stream()
            check(lib().bicgstab_update_values(self._h, C.c_void_p(self.values.data_ptr())),
                  "bicgstab_update_values")
        self.values_version += 1

    def spmm(self, X, out=None):
        X = self._block(X, "X")
        Y = torch.empty_like(X) if out is None else out
        with torch.cuda.device(self.device):
            self._set_stream()
            check(lib().bicgstab_spmm(self._h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr())), "bicgstab_spmm")
        return Y

    def product_layout(self):
        """(tile (tz, ty, tx), grid (nz, ny, nx)) of the tile-ordered storage the
        plain product uses, or zeros when A is stored row by row."""
        t = (C.c_int32 * 3)()
        g = (C.c_int32 * 3)()
        check(lib().bicgstab_product_layout(self._h, t, g), "bicgstab_product_layout")
        return tuple(t), tuple(g)

    def history(self):
        """(iterations, k, 4) array of alpha, omega, rho, stop estimate."""
        cnt = C.c_int32()
        L = lib()
        check(L.bicgstab_history(self._h, None, 0, C.byref(cnt)), "bicgstab_history")
        m = cnt.value
        buf = np.zeros(max(m, 1) * self.k * 4, np.float64)
        check(L.bicgstab_history(self._h, buf.ctypes.data_as(C.POINTER(C.c_double)), m * self.k, C.byref(cnt)),
              "bicgstab_history")
        return buf[: cnt.value * self.k * 4].reshape(cnt.value, self.k, 4)

    def refine_outer(self):
        """FP32-refinement handles: FP64 corrections applied per column."""
        out = np.zeros(self.k, np.int32)
        check(lib().bicgstab_refine_outer(self._h, out.ctypes.data_as(C.POINTER(C.c_int32))), "bicgstab_refine_outer")
        return out

    def stats(self):
        a, b_, c = C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().bicgstab_last_solve_stats(self._h, C.byref(a), C.byref(b_), C.byref(c)), "stats")
        return {"iterations_enqueued": a.value, "launches": b_.value, "polls": c.value}

    def kernel_times(self, b, x, iters: int = 10):
        """Per-kernel average duration (ms) of one iteration's launches, timed
        with HIP events around each launch on the stream it runs on."""
        L = lib()
        b = self._block(b, "b")
        x = self._block(x, "x")
        cap = 64
        kind, op, nin, nout = (np.zeros(cap, np.int32) for _ in range(4))
        ms = np.zeros(cap, np.float64)
        ns = C.c_int32()
        P = C.POINTER(C.c_int32)
        with torch.cuda.device(self.device):
            self._set_stream()
            check(L.bicgstab_kernel_times(self._h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), int(iters), cap,
                                          kind.ctypes.data_as(P), op.ctypes.data_as(P), nin.ctypes.data_as(P),
                                          nout.ctypes.data_as(P), ms.ctypes.data_as(C.POINTER(C.c_double)),
                                          C.byref(ns)), "bicgstab_kernel_times")
        m = ns.value
        return [{"kind": ["spmm", "prec", "group", "spmm_dot"][kind[i]], "op": int(op[i]), "nin": int(nin[i]),
                 "nout": int(nout[i]), "ms": float(ms[i])} for i in range(m)]

    def close(self):
        if getattr(self, "_h", None):
            lib().bicgstab_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_traffic(variant: str, formulation: str, precond: str):
    """Per-iteration vector reads/writes, preconditioner applications, sparse
    products and launches of a method's launch plan (host-only query)."""
    L = lib()
    v = [C.c_int32() for _ in range(5)]
    check(L.bicgstab_plan_traffic(_lib.VARIANTS[variant], _lib.FORMULATIONS[formulation], _lib.PRECONDS[precond],
                                  *[C.byref(x) for x in v]), "bicgstab_plan_traffic")
    r, w, p, s, l = (x.value for x in v)
    return {"reads": r, "writes": w, "precond_apps": p, "spmms": s, "launches": l}


def axpby_tab1(run: int, x, y, z, a: float, b: float, c: float):
    """Table 1's vector updates on device tensors (float64, same length; y and
    z updated in place): run 1 as three passes, run 2 the first two updates
    merged, run 3 all three merged. Enqueued on torch's current stream."""
    n = int(x.numel())
    for t, name in ((x, "x"), (y, "y"), (z, "z")):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or int(t.numel()) != n:
            raise ValueError(f"{name} must be a contiguous float64 device tensor of length {n}")
    with torch.cuda.device(x.device):
        check(lib().bicgstab_axpby_tab1(int(run), n, float(a), float(b), float(c), C.c_void_p(x.data_ptr()),
                                        C.c_void_p(y.data_ptr()), C.c_void_p(z.data_ptr()),
                                        C.c_void_p(_stream_ptr(x.device))), "bicgstab_axpby_tab1")
