"""Batched tier front end: many independent sparse systems of uneven size
solved by one persistent kernel launch of the HIP library (argument
marshalling only; every step runs in the library's kernels)."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import check, lib
from .solver import SolveInfo, _dev_tensor, _stream_ptr


@dataclass
class BatchedConfig:
    variant: int  # kernel variant index (variant_info)
    block: int  # threads per workgroup
    workgroups: np.ndarray  # share of each system
    last_ms: float  # kernel time of the last solve
    system_ms: np.ndarray  # device wall time of each system in the last solve


def variant_info(variant: int):
    """(threads per workgroup, rows per vector-phase step, entries per
    pipelined row-product step, rows per stage of the sparse products'
    pipeline)."""
    b, r, e, pr = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
    check(lib().bicgstab_batched_variant_info(int(variant), C.byref(b), C.byref(r), C.byref(e), C.byref(pr)),
          "bicgstab_batched_variant_info")
    return int(b.value), int(r.value), int(e.value), int(pr.value)


class BatchedSolver:
    """systems: a sequence of (row_ptr, col_idx, values, k) or of (A, k) with A
    a host CSR object (row_ptr / col_idx / values arrays). precond: "none" or
    "jacobi" (every system; the classical method in either case)."""

    def __init__(self, systems, device="cuda", precond="none"):
        self.device = torch.device(device)
        self._mats = []
        descs, ks = [], []
        for item in systems:
            if len(item) == 2:
                A, k = item
                rp, ci, va = A.row_ptr, A.col_idx, A.values
            else:
                rp, ci, va, k = item
            rp = _dev_tensor(np.asarray(rp, dtype=np.int32), torch.int32, self.device, "row_ptr")
            ci = _dev_tensor(np.asarray(ci, dtype=np.int32), torch.int32, self.device, "col_idx")
            va = _dev_tensor(np.asarray(va, dtype=np.float64), torch.float64, self.device, "values")
            self._mats.append((rp, ci, va))
            n = int(rp.numel()) - 1
            descs.append(_lib.CSRDesc(n, int(ci.numel()), rp.data_ptr(), ci.data_ptr(), va.data_ptr()))
            ks.append(int(k))
        self.nsys = len(descs)
        self.n = [d.n for d in descs]
        self.k = ks
        arr = (_lib.CSRDesc * self.nsys)(*descs)
        karr = (C.c_int32 * self.nsys)(*ks)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().bicgstab_batched_create(arr, karr, self.nsys, _lib.VARIANTS["classical"],
                                                _lib.PRECONDS[precond], C.c_void_p(_stream_ptr(self.device)),
                                                C.byref(h)), "bicgstab_batched_create")
        self._h = h
        nbytes = C.c_size_t()
        check(lib().bicgstab_batched_workspace_bytes(h, C.byref(nbytes)), "bicgstab_batched_workspace_bytes")
        self.workspace = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=self.device)
        check(lib().bicgstab_batched_set_workspace(h, C.c_void_p(self.workspace.data_ptr()), self.workspace.numel()),
              "bicgstab_batched_set_workspace")

    def _blocks(self, ts, name):
        if len(ts) != self.nsys:
            raise ValueError(f"{name}: {self.nsys} blocks expected, got {len(ts)}")
        out = []
        for s, t in enumerate(ts):
            t = _dev_tensor(t, torch.float64, self.device, name)
            if t.dim() == 1:
                t = t.view(-1, 1)
            if tuple(t.shape) != (self.n[s], self.k[s]):
                raise ValueError(f"{name}[{s}] must be {self.n[s]} x {self.k[s]}, got {tuple(t.shape)}")
            out.append(t)
        return out

    def _ptrs(self, ts):
        return (C.c_void_p * self.nsys)(*[t.data_ptr() for t in ts])

    def _prepare(self, bs, x0s):
        bs = self._blocks(bs, "b")
        if x0s is None:
            xs = [torch.zeros_like(b) for b in bs]
        else:
            xs = [x.clone() for x in self._blocks(x0s, "x0")]
        return bs, xs

    def solve(self, bs, x0s=None, tol: float = 1e-8, maxit: int = 1000):
        """Solve every system. Returns (list of X_s, list of SolveInfo)."""
        bs, xs = self._prepare(bs, x0s)
        tc = sum(self.k)
        arrs = (np.zeros(tc, np.int32), np.zeros(tc, np.int32), np.zeros(tc, np.float64), np.zeros(tc, np.float64))
        info = _lib.Info(arrs[0].ctypes.data_as(C.POINTER(C.c_int32)), arrs[1].ctypes.data_as(C.POINTER(C.c_int32)),
                         arrs[2].ctypes.data_as(C.POINTER(C.c_double)), arrs[3].ctypes.data_as(C.POINTER(C.c_double)))
        with torch.cuda.device(self.device):
            check(lib().bicgstab_batched_set_stream(self._h, C.c_void_p(_stream_ptr(self.device))),
                  "bicgstab_batched_set_stream")
            check(lib().bicgstab_batched_solve(self._h, self._ptrs(bs), self._ptrs(xs), float(tol), int(maxit),
                                               C.byref(info)), "bicgstab_batched_solve")
        infos, c0 = [], 0
        for k in self.k:
            infos.append(SolveInfo(*(a[c0:c0 + k].copy() for a in arrs)))
            c0 += k
        return xs, infos

    def tune(self, bs, x0s=None, tol: float = 1e-8, maxit: int = 1000):
        """Run the autotuner on this batch; returns (best kernel ms, list of X_s)."""
        bs, xs = self._prepare(bs, x0s)
        best = C.c_double()
        with torch.cuda.device(self.device):
            check(lib().bicgstab_batched_set_stream(self._h, C.c_void_p(_stream_ptr(self.device))),
                  "bicgstab_batched_set_stream")
            check(lib().bicgstab_batched_tune(self._h, self._ptrs(bs), self._ptrs(xs), float(tol), int(maxit),
                                              C.byref(best)), "bicgstab_batched_tune")
        return best.value, xs

    def config(self):
        """BatchedConfig of the current configuration and the last solve."""
        var, blk = C.c_int32(), C.c_int32()
        wg = (C.c_int32 * self.nsys)()
        ms = C.c_double()
        sms = (C.c_double * self.nsys)()
        check(lib().bicgstab_batched_get_config(self._h, C.byref(var), C.byref(blk), wg, C.byref(ms), sms),
              "bicgstab_batched_get_config")
        return BatchedConfig(int(var.value), int(blk.value), np.array(wg[:], dtype=np.int32), float(ms.value),
                             np.array(sms[:]))

    def set_config(self, variant: int, workgroups):
        wg = (C.c_int32 * self.nsys)(*[int(v) for v in workgroups])
        check(lib().bicgstab_batched_set_config(self._h, int(variant), wg), "bicgstab_batched_set_config")

    def close(self):
        if getattr(self, "_h", None):
            lib().bicgstab_batched_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
