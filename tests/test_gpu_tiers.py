"""GPU tests of the precision tier (FP32 inner solves + FP64 refinement) and
the differentiation tier (adjoint solve with A^T, pattern-restricted
gradient, torch.autograd chaining), against the CPU oracle, dense autograd
and finite differences."""
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import adjoint as oad
from oracle import refine as orf
from workloads import conv_diff, manufactured_rhs, random_27pt
from workloads import generators as wg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ------------------------------------------------------------- precision ---

@pytest.mark.parametrize("variant,precond,formulation", [("classical", "none", "merged"), ("classical", "jacobi", "merged"),
                                                         ("pipelined", "none", "merged"), ("pipelined", "jacobi", "merged"),
                                                         ("reordered", "jacobi", "merged"), ("classical", "jacobi", "fused"),
                                                         ("reordered", "jacobi", "fused"), ("pipelined", "none", "fused"),
                                                         ("pipelined", "jacobi", "fused")])
def test_precision_tier_matches_refinement_oracle(lib, variant, precond, formulation):
    """27-point random matrix (the precision-tier recipe at 20^3), k = 8,
    tol 1e-10: every column converges in FP64 terms, the number of FP64
    corrections matches the NumPy FP32-refinement oracle within 1, and the
    error against a tight FP64 solve is within the conditioning bound."""
    import torch

    say(f"precision tier {variant}/{precond}/{formulation}")
    A = random_27pt(20, seed=3)
    S = A.to_scipy()
    b, xs = manufactured_rhs(A, 8, seed=4)
    s = lib.Solver.from_csr(A, 8, variant=variant, formulation=formulation, precond=precond, precision="fp32_refine")
    x, info = s.solve(torch.from_numpy(b).cuda(), tol=1e-10, maxit=5000)
    X = x.cpu().numpy()
    outer = s.refine_outer()
    assert np.all(info.status == 0), info.status
    rt = np.linalg.norm(b - S @ X, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(rt < 1e-10) and np.allclose(rt, info.relres_true, rtol=1e-6)
    tight = oracle.solve(S, b, tol=1e-13, maxit=5000)
    nt = np.linalg.norm(tight.x, axis=0)
    err = np.linalg.norm(X - tight.x, axis=0) / nt
    # equal accuracy: the FP64 solve to the same tolerance on the same GPU
    s64 = lib.Solver.from_csr(A, 8, variant=variant, formulation=formulation, precond=precond)
    x64, info64 = s64.solve(torch.from_numpy(b).cuda(), tol=1e-10, maxit=5000)
    err64 = np.linalg.norm(x64.cpu().numpy() - tight.x, axis=0) / nt
    say(f"  outer {list(outer)}, max rel error vs FP64 tight solve {err.max():.2e} (FP64 solve at the same tol "
        f"{err64.max():.2e})")
    assert np.all(err <= 5 * err64 + 1e-10), (err, err64)
    # refined further, the solution error itself falls below 1e-10
    x12, info12 = s.solve(torch.from_numpy(b).cuda(), tol=1e-12, maxit=5000)
    err12 = np.linalg.norm(x12.cpu().numpy() - tight.x, axis=0) / nt
    say(f"  refined to 1e-12: outer {list(s.refine_outer())}, max rel error {err12.max():.2e}")
    assert np.all(info12.status == 0) and np.all(err12 < 1e-10)
    if variant == "classical":
        for c in range(8):
            ref = orf.refine_solve(S, b[:, c], tol=1e-10, inner_tol=1e-5, precond=precond)
            assert ref["status"] == oracle.CONVERGED
            assert abs(int(outer[c]) - ref["outer"]) <= 1, (c, outer[c], ref["outer"])


@pytest.mark.parametrize("k", [3, 6, 4])
def test_precision_tier_edge_columns(lib, k):
    """A zero right-hand side column and a nonzero x0 in the FP32 tier, for
    the three FP32 product layouts (k = 3: one column per lane, 6: two, 4:
    four): every column converges in FP64 terms, the zero column stays 0."""
    import torch

    say(f"precision tier edges k={k}")
    A = conv_diff(8, 3, (1.0, 0.7, 0.3))
    n = A.n
    b, _ = manufactured_rhs(A, k, seed=5)
    b[:, 1] = 0.0
    s = lib.Solver.from_csr(A, k, precision="fp32_refine")
    x0 = torch.ones(n, k, dtype=torch.float64).cuda()
    x, info = s.solve(torch.from_numpy(b).cuda(), x0, tol=1e-10, maxit=2000)
    X = x.cpu().numpy()
    assert list(info.status) == [0] * k
    assert np.all(X[:, 1] == 0)
    others = [c for c in range(k) if c != 1]
    assert np.all(info.relres_true[others] < 1e-10)
    rt = np.linalg.norm(b - A.to_scipy() @ X, axis=0)[others] / np.linalg.norm(b, axis=0)[others]
    assert np.all(rt < 1e-10)


# --------------------------------------------------------- differentiation ---

def test_grad_values_kernel(lib):
    """The SDDMM kernel against the pattern-gradient definition."""
    import torch

    say("grad_values kernel")
    A = conv_diff(11, 3, (1.0, -0.5, 0.25))
    for k in (1, 3, 8, 32):
        rng = np.random.default_rng(k)
        lam = rng.uniform(-1, 1, (A.n, k))
        X = rng.uniform(-1, 1, (A.n, k))
        s = lib.Solver.from_csr(A, k)
        g = s.grad_values(torch.from_numpy(lam).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
        ref = oad.pattern_grad(A.to_scipy(), lam, X)
        scale = np.abs(lam)[A.row_of_entry()].sum(axis=1) * 1.0 + 1e-300
        assert np.all(np.abs(g - ref) <= 16 * np.finfo(float).eps * scale * max(1, k))


@pytest.mark.parametrize("variant,precond,formulation", [("classical", "none", "merged"), ("classical", "jacobi", "merged"),
                                                         ("classical", "jacobi", "fused"), ("improved", "none", "merged"),
                                                         ("reordered", "jacobi", "fused"), ("reordered", "none", "fused"),
                                                         ("pipelined", "jacobi", "merged"), ("pipelined", "jacobi", "fused")])
def test_transpose_solve(lib, variant, precond, formulation):
    """A^T Lambda = G by the same method on the device-built transposed CSR
    (nonsymmetric matrix, so A vs A^T matters)."""
    import torch

    say(f"transpose solve {variant} {precond} {formulation}")
    A = conv_diff(14, 3, (3.0, -2.0, 1.5))
    St = A.to_scipy().T.tocsr()
    G = np.random.default_rng(11).uniform(-1, 1, (A.n, 4))
    s = lib.Solver.from_csr(A, 4, variant=variant, precond=precond, formulation=formulation)
    lam, info = s.solve_transpose(torch.from_numpy(G).cuda(), tol=1e-12, maxit=3000)
    L = lam.cpu().numpy()
    assert np.all(info.status == 0)
    rt = np.linalg.norm(G - St @ L, axis=0) / np.linalg.norm(G, axis=0)
    assert np.all(rt < 1.1e-12)
    ref = np.linalg.solve(St.toarray(), G)
    assert np.linalg.norm(L - ref) / np.linalg.norm(ref) < 1e-9


def _dense_grad_field(A, assemble, field, B):
    import torch

    rows = torch.as_tensor(A.row_of_entry())
    cols = torch.as_tensor(A.col_idx.astype(np.int64))
    ft = torch.tensor(field, dtype=torch.float64, requires_grad=True)
    vals = assemble(ft)
    Ad = torch.zeros(A.n, A.n, dtype=torch.float64).index_put((rows, cols), vals)
    X = torch.linalg.solve(Ad, torch.as_tensor(B))
    (X * X).sum().backward()
    return ft.grad.numpy()


def test_autograd_diffusion_12cubed(lib):
    """The differentiation-tier recipe at 12^3 (k = 8): gradient of
    sum ||x||^2 with respect to the log-conductivity field through the GPU
    solve and adjoint, against torch autograd of a dense FP64 solve, and
    against central differences of GPU solves."""
    import torch

    from paper_1907_12874_amd import autograd as pag

    say("autograd 12^3")
    g0 = 12
    A, field = wg.diffusion_varcoef(g0, seed=0)
    B = np.random.default_rng(7).uniform(-1, 1, (A.n, 8))
    assemble = wg.diffusion_values_torch(A, g0)
    s = lib.Solver.from_csr(A, 8)
    ft = torch.tensor(field, dtype=torch.float64, device="cuda", requires_grad=True)
    Bt = torch.from_numpy(B).cuda()
    X = pag.solve(assemble(ft), Bt, s, tol=1e-13, maxit=3000)
    (X * X).sum().backward()
    grad = ft.grad.cpu().numpy()
    ref = _dense_grad_field(A, assemble, field, B)
    assert np.linalg.norm(grad - ref) / np.linalg.norm(ref) < 1e-8

    def loss(fld):
        with torch.no_grad():
            Xl = pag.solve(assemble(torch.from_numpy(fld).cuda()), Bt, s, tol=1e-13, maxit=3000)
            return float((Xl * Xl).sum())

    # iterative solves at 1e-13 leave ~1e-10 relative noise in the loss, so the
    # step is 1e-4 (central-difference truncation ~1e-8) and the bar 2e-5
    rng = np.random.default_rng(12)
    h = 1e-4
    for _ in range(3):
        d = rng.standard_normal(A.n)
        fd = (loss(field + h * d) - loss(field - h * d)) / (2 * h)
        an = grad @ d
        assert abs(fd - an) <= 2e-5 * abs(an), (fd, an)


def test_autograd_nonsymmetric_values_and_b(lib):
    """Nonsymmetric matrix: gradients with respect to the stored values and
    to B against dense autograd (catches A vs A^T mix-ups)."""
    import torch

    from paper_1907_12874_amd import autograd as pag

    say("autograd nonsymmetric")
    A = conv_diff(6, 3, (3.0, -2.0, 1.5))
    B = np.random.default_rng(13).uniform(-1, 1, (A.n, 3))
    s = lib.Solver.from_csr(A, 3)
    v = torch.tensor(A.values, dtype=torch.float64, device="cuda", requires_grad=True)
    Bt = torch.tensor(B, dtype=torch.float64, device="cuda", requires_grad=True)
    X = pag.solve(v, Bt, s, tol=1e-13, maxit=3000)
    w = torch.linspace(-1, 1, X.numel(), dtype=torch.float64, device="cuda").view_as(X)
    ((X * X).sum() + (w * X).sum()).backward()
    rows = torch.as_tensor(A.row_of_entry())
    cols = torch.as_tensor(A.col_idx.astype(np.int64))
    vc = torch.tensor(A.values, dtype=torch.float64, requires_grad=True)
    Bc = torch.tensor(B, dtype=torch.float64, requires_grad=True)
    Ad = torch.zeros(A.n, A.n, dtype=torch.float64).index_put((rows, cols), vc)
    Xc = torch.linalg.solve(Ad, Bc)
    ((Xc * Xc).sum() + (w.cpu() * Xc).sum()).backward()
    gv, gb = v.grad.cpu().numpy(), Bt.grad.cpu().numpy()
    assert np.linalg.norm(gv - vc.grad.numpy()) / np.linalg.norm(vc.grad.numpy()) < 1e-9
    assert np.linalg.norm(gb - Bc.grad.numpy()) / np.linalg.norm(Bc.grad.numpy()) < 1e-9


def test_autograd_full_size_64cubed(lib):
    """The 64^3 diffusion workload, k = 8: forward and backward converge and
    the directional derivative of the loss along a random field direction
    matches a central difference of GPU solves."""
    import torch

    from paper_1907_12874_amd import autograd as pag

    say("autograd 64^3")
    cfg = wg.config_problem(4, seed=0)
    A, field, B = cfg["A"], cfg["field"], cfg["b"]
    assemble = wg.diffusion_values_torch(A, cfg["g"])
    s = lib.Solver.from_csr(A, 8)
    Bt = torch.from_numpy(B).cuda()
    ft = torch.tensor(field, dtype=torch.float64, device="cuda", requires_grad=True)
    X = pag.solve(assemble(ft), Bt, s, tol=1e-12, maxit=5000)
    (X * X).sum().backward()
    grad = ft.grad.cpu().numpy()
    d = np.random.default_rng(14).standard_normal(A.n)
    h = 1e-4

    def loss(fld):
        with torch.no_grad():
            Xl = pag.solve(assemble(torch.from_numpy(fld).cuda()), Bt, s, tol=1e-12, maxit=5000)
            return float((Xl * Xl).sum())

    fd = (loss(field + h * d) - loss(field - h * d)) / (2 * h)
    an = grad @ d
    assert abs(fd - an) <= 1e-4 * abs(an), (fd, an)


def test_autograd_solver_reused_before_backward(lib):
    """One solver, two differentiable solves with different matrix values
    before either backward runs (two solves in one loss): each gradient
    equals dense FP64 autograd of its own solve, so the adjoint of the first
    solve runs with the first solve's A^T, not the values the solver held
    last."""
    import torch

    from paper_1907_12874_amd import autograd as pag

    say("autograd: one solver, two forwards, then backward")
    A = conv_diff(6, 3, (3.0, -2.0, 1.5))
    B = np.random.default_rng(17).uniform(-1, 1, (A.n, 2))
    s = lib.Solver.from_csr(A, 2)
    rows = torch.as_tensor(A.row_of_entry())
    cols = torch.as_tensor(A.col_idx.astype(np.int64))
    scales = (1.0, 1.7)
    vs = [torch.tensor(A.values * sc, dtype=torch.float64, device="cuda", requires_grad=True) for sc in scales]
    Bt = torch.from_numpy(B).cuda()
    X1 = pag.solve(vs[0], Bt, s, tol=1e-13, maxit=3000)
    X2 = pag.solve(vs[1], Bt, s, tol=1e-13, maxit=3000)
    w = torch.linspace(-1, 1, X1.numel(), dtype=torch.float64, device="cuda").view_as(X1)
    # the first solve's backward alone, while the solver holds the second's values
    ((X1 * X1).sum() + (w * X1).sum()).backward(retain_graph=True)
    g1 = vs[0].grad.cpu().numpy().copy()
    (X2 * X2).sum().backward()
    g2 = vs[1].grad.cpu().numpy().copy()
    for sc, g, extra in ((scales[0], g1, True), (scales[1], g2, False)):
        vc = torch.tensor(A.values * sc, dtype=torch.float64, requires_grad=True)
        Ad = torch.zeros(A.n, A.n, dtype=torch.float64).index_put((rows, cols), vc)
        Xc = torch.linalg.solve(Ad, torch.from_numpy(B))
        loss = (Xc * Xc).sum() + ((w.cpu() * Xc).sum() if extra else 0.0)
        loss.backward()
        ref = vc.grad.numpy()
        assert np.linalg.norm(g - ref) / np.linalg.norm(ref) < 1e-9, (sc, np.linalg.norm(g - ref) / np.linalg.norm(ref))


def test_update_values_with_a_new_array(lib):
    """bicgstab_update_values through the C ABI: handing the handle another
    values array (same pattern) gives the solve of a handle created on that
    array, bit for bit, Jacobi diagonal included; a NULL pointer after an
    in-place change of the borrowed array does the same."""
    import ctypes as C

    import torch

    from paper_1907_12874_amd import _lib

    say("update_values with a new array / NULL after an in-place change")
    A = conv_diff(12, 3, (0.5, -0.3, 0.2))
    k = 3
    b = torch.from_numpy(manufactured_rhs(A, k, seed=4)[0]).cuda()
    vals2 = A.values * 1.25
    vals2[A.col_idx == A.row_of_entry()] *= 1.1  # a different diagonal
    A2 = wg.CSR(A.n, A.row_ptr, A.col_idx, vals2)
    s = lib.Solver.from_csr(A, k, precond="jacobi")
    x1, _ = s.solve(b, tol=1e-10, maxit=1000)
    v2 = torch.from_numpy(vals2).cuda()
    L = _lib.lib()
    assert L.bicgstab_update_values(s._h, C.c_void_p(v2.data_ptr())) == 0
    x2, info2 = s.solve(b, tol=1e-10, maxit=1000)
    ref = lib.Solver.from_csr(A2, k, precond="jacobi")
    xr, infor = ref.solve(b, tol=1e-10, maxit=1000)
    assert np.array_equal(info2.iters, infor.iters)
    assert torch.equal(x2, xr)
    assert not torch.equal(x1, x2)
    # in place on the array the handle now borrows, then NULL
    v2.mul_(0.8)
    assert L.bicgstab_update_values(s._h, None) == 0
    x3, _ = s.solve(b, tol=1e-10, maxit=1000)
    ref3 = lib.Solver.from_csr(wg.CSR(A.n, A.row_ptr, A.col_idx, vals2 * 0.8), k, precond="jacobi")
    xr3, _ = ref3.solve(b, tol=1e-10, maxit=1000)
    assert torch.equal(x3, xr3)
    s.close()
    ref.close()
    ref3.close()
    del v2


def test_precision_tier_inner_trajectory_full_size(lib):
    """The precision tier's first FP32 inner solve at full size (27-point
    random 100^3, k = 32), stopped after 15 inner passes (the inner solve to
    1e-5 takes 17), on columns 0 and 31: x = ||b_c|| d_15 equals, bit for
    bit, the refinement oracle's FP32
    inner solve (oracle.refine.inner_merged_fp32) run with the kernels'
    dot-product summation order. FP32 storage, FP32-accumulated products,
    FP64 dots and scalars and the FP64 inner solution d all round the same
    way on both sides."""
    import math

    import torch

    sys.path.insert(0, os.path.join(os.path.dirname(__file__)))
    from kernel_order import group_dot

    say("precision tier: 15 inner FP32 passes at 100^3, k = 32 (bitwise)")
    from workloads import config_problem

    cfg = config_problem(2, seed=0)
    A, b, k = cfg["A"], cfg["b"], cfg["k"]
    s = lib.Solver.from_csr(A, k, precision="fp32_refine")
    x, info = s.solve(torch.from_numpy(b).cuda(), tol=1e-10, maxit=15)
    X = x.cpu().numpy()
    S = A.to_scipy()
    A32 = S.astype(np.float32)
    g = group_dot(A.n, k)
    saved = orf._dot
    # the inner solve's dots accumulate FP64 products of FP32 operands
    orf._dot = lambda u, w: g(np.asarray(u, np.float64), np.asarray(w, np.float64))
    try:
        for c in (0, k - 1):
            r = b[:, c] - S @ np.zeros(A.n)  # r = b - A x0 with x0 = 0
            scale = math.sqrt(g(r, r))
            d, passes, _ = orf.inner_merged_fp32(A32, None, (r / scale).astype(np.float32), 1e-5, 15)
            assert passes == int(info.iters[c]) == 15
            assert np.array_equal(X[:, c], 0.0 + scale * d), (c, np.abs(X[:, c] - scale * d).max())
    finally:
        orf._dot = saved
    s.close()


def test_precision_tier_error_vs_fp64_oracle_full_size(lib):
    """The precision tier's workload at full size (27-point random 100^3,
    k = 32, tol 1e-10): FP32 inner solves with FP64 refinement and the plain
    FP64 solve on the same GPU, each against the CPU FP64 oracle run to
    1e-12 on columns 0 and 31. The refined solution's error is stated and
    stays within 5x that of the FP64 solve to the same tolerance; refined
    further, to a residual of 1e-12, it falls below 1e-10."""
    import torch

    from workloads import config_problem

    say("precision tier: error against the FP64 oracle at 100^3, k = 32")
    cfg = config_problem(2, seed=0)
    A, b, k = cfg["A"], cfg["b"], cfg["k"]
    S = A.to_scipy()
    bt = torch.from_numpy(b).cuda()
    out = {}
    for prec in ("fp32_refine", "fp64"):
        s = lib.Solver.from_csr(A, k, precision=prec)
        x, info = s.solve(bt, tol=1e-10, maxit=5000)
        assert np.all(info.status == 0)
        out[prec] = x.cpu().numpy()
        s.close()
    errs = {p: [] for p in out}
    refs = []
    for c in (0, k - 1):
        ref = oracle.solve_column(S, b[:, c], None, "classical", "merged", "none", 1e-12, 5000)
        assert ref.status == oracle.CONVERGED
        refs.append(ref)
        nr = np.linalg.norm(ref.x)
        for p in out:
            errs[p].append(float(np.linalg.norm(out[p][:, c] - ref.x) / nr))
    say(f"  relative error vs the FP64 oracle (tol 1e-12), columns 0 and {k - 1}: FP32+refinement "
        f"{errs['fp32_refine']}, FP64 {errs['fp64']}")
    for e32, e64 in zip(errs["fp32_refine"], errs["fp64"]):
        assert e32 <= 5 * e64 + 1e-10
    # the error itself below 1e-10: refined to a residual of 1e-12
    s = lib.Solver.from_csr(A, k, precision="fp32_refine")
    x, info = s.solve(bt, tol=1e-12, maxit=5000)
    assert np.all(info.status == 0)
    X = x.cpu().numpy()
    s.close()
    tight = [float(np.linalg.norm(X[:, c] - r.x) / np.linalg.norm(r.x)) for c, r in zip((0, k - 1), refs)]
    say(f"  FP32+refinement to a residual of 1e-12: error vs the oracle {tight}")
    assert max(tight) < 1e-10
