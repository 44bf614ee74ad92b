"""The allocation-free solve (bicgstab_solve_noalloc) against bicgstab_solve,
through the C ABI: bitwise the same solutions, pass counts, statuses and
residuals, on two calls in a row (the second with a smaller system, which
finds the first call's contents in the shared static scratch), and the size
limit reported as an error."""
import sys

import numpy as np
import pytest

from workloads import conv_diff, manufactured_rhs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [("classical", "merged", "jacobi"), ("classical", "basic", "none"), ("classical", "fused", "jacobi"),
         ("reordered", "merged", "jacobi"), ("reordered", "fused", "jacobi"), ("pipelined", "merged", "jacobi"),
         ("pipelined", "basic", "none")]


@pytest.mark.parametrize("variant,formulation,precond", CASES)
def test_noalloc_equals_solve_two_calls(lib, variant, formulation, precond):
    import torch

    systems = [(conv_diff(24, 3, (1.0, 0.7, 0.3)), 5, 0), (conv_diff(16, 2, (1.0, 0.5)), 2, 1)]
    for A, k, seed in systems:  # the second call is the smaller one
        say(f"noalloc {variant}/{formulation}/{precond} n={A.n} k={k}")
        b = torch.from_numpy(manufactured_rhs(A, k, seed=seed)[0]).cuda()
        s = lib.Solver.from_csr(A, k, variant=variant, formulation=formulation, precond=precond)
        x_ref, i_ref = s.solve(b, tol=1e-10, maxit=2000)
        x_na, i_na = s.solve_noalloc(b, tol=1e-10, maxit=2000)
        torch.cuda.synchronize()
        assert np.array_equal(i_na.iters, i_ref.iters), (i_na.iters, i_ref.iters)
        assert np.array_equal(i_na.status, i_ref.status), (i_na.status, i_ref.status)
        assert np.array_equal(i_na.relres_true, i_ref.relres_true)
        assert np.array_equal(i_na.relres_recursive, i_ref.relres_recursive)
        assert torch.equal(x_na, x_ref)
        assert np.all(i_ref.status == 0)
        # the handle's own workspace is untouched: a normal solve after the
        # allocation-free one is unchanged
        x_again, i_again = s.solve(b, tol=1e-10, maxit=2000)
        assert torch.equal(x_again, x_ref) and np.array_equal(i_again.iters, i_ref.iters)
        s.close()


def test_noalloc_limits(lib):
    """A handle whose workspace exceeds the static scratch, Improved BiCGStab
    and the FP32 tier are refused with an error; the library stays usable."""
    import torch

    from paper_1907_12874_amd._lib import BicgstabError, ENOMEM, EUNSUPPORTED

    say("noalloc limits")
    A = conv_diff(64, 3, (1.0, 0.7, 0.3))  # 262,144 rows: 64 columns need far more than 64 MiB
    s = lib.Solver.from_csr(A, 64, precond="jacobi")
    b = torch.ones(A.n, 64, dtype=torch.float64, device="cuda")
    with pytest.raises(BicgstabError) as e:
        s.solve_noalloc(b, tol=1e-8, maxit=10)
    assert e.value.code == ENOMEM
    s.close()
    B = conv_diff(10, 2, (1.0, 0.5))
    for kw in ({"variant": "improved"}, {"precision": "fp32_refine"}):
        s = lib.Solver.from_csr(B, 1, **kw)
        with pytest.raises(BicgstabError) as e:
            s.solve_noalloc(torch.ones(B.n, 1, dtype=torch.float64, device="cuda"), tol=1e-8, maxit=10)
        assert e.value.code == EUNSUPPORTED
        s.close()
    # and a regular small solve still works afterwards
    s = lib.Solver.from_csr(B, 1)
    x, info = s.solve_noalloc(torch.ones(B.n, 1, dtype=torch.float64, device="cuda"), tol=1e-10, maxit=500)
    assert np.all(info.status == 0)
    s.close()
