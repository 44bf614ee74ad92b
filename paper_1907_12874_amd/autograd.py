"""Differentiable multi-RHS solve: X = A(values)^{-1} B as a torch.autograd.Function.

Forward: the library's BiCGStab on A. Backward (hand-written adjoint):
Lambda = A^{-T} dL/dX by the same BiCGStab on the transposed CSR (built on the
device at first use), dL/dB = Lambda, and dL/dvalues[e] = -sum_c Lambda[i,c]
X[j,c] for every stored entry e = (i, j) (one kernel). Every step runs in the
library's kernels; this module only passes tensors.
"""
from __future__ import annotations

import torch

from .solver import Solver


class BicgstabSolve(torch.autograd.Function):
    """apply(values, B, solver, tol, maxit) -> X. `solver` is a Solver built
    on the same sparsity pattern; its values are replaced by `values`.

    One solver may serve several forwards before their backwards run (two
    solves in one loss, recomputation): each forward keeps its own values and
    the solver's value version, and its backward puts those values back into
    the solver first if another forward (or any update_values) has replaced
    them since, so the adjoint solve always uses this forward's A^T."""

    @staticmethod
    def forward(ctx, values, B, solver: Solver, tol: float, maxit: int):
        vals = values.detach()
        solver.update_values(vals)
        X, info = solver.solve(B.detach(), tol=tol, maxit=maxit)
        if not info.converged:
            raise RuntimeError(f"forward solve did not converge: status {info.status}")
        ctx.solver, ctx.tol, ctx.maxit = solver, tol, maxit
        ctx.version = solver.values_version
        # a private copy: the caller may change `values` in place after the
        # forward, and the adjoint must see the matrix that produced X
        ctx.save_for_backward(X, vals.clone())
        return X

    @staticmethod
    def backward(ctx, gX):
        X, vals = ctx.saved_tensors
        s = ctx.solver
        if s.values_version != ctx.version:
            s.update_values(vals)
            ctx.version = s.values_version
        lam, info = s.solve_transpose(gX.contiguous(), tol=ctx.tol, maxit=ctx.maxit)
        if not info.converged:
            raise RuntimeError(f"adjoint solve did not converge: status {info.status}")
        gvals = s.grad_values(lam, X) if ctx.needs_input_grad[0] else None
        gB = lam if ctx.needs_input_grad[1] else None
        return gvals, gB, None, None, None


def solve(values, B, solver: Solver, tol: float = 1e-10, maxit: int = 5000):
    """Differentiable X = A(values)^{-1} B."""
    return BicgstabSolve.apply(values, B, solver, tol, maxit)
