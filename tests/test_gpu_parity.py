"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.

Bitwise. Every dot product of the non-fused plans is formed by the vector-pass
kernel and the finalize kernel in a fixed order that depends only on n, k and
the pass's grid; run with its dot product summed in that order
(`kernel_order.group_dot`), the oracle reproduces the library's trajectories
and converged solves bit for bit: pass counts, statuses, per-pass scalars and
iterates (`test_bitwise_*`). The envelope tests below compare against the
oracle's own summation order instead.

Tolerances. The library evaluates every vector update and sparse product in
the same order as the oracle with no fused multiply-add, and divides by a_ii
for Jacobi, so those steps round identically; only the dot products sum in a
different order (a fixed tree on the GPU, BLAS on the CPU). BiCGStab
amplifies that difference as the residual falls, and by the same amount for
any two summation orders, so the bars are measured, not guessed: the oracle is
rerun with its dot products summed in three other orders, and the spread of
those runs is the envelope the GPU must stay inside.
  * sparse products: bitwise equal to SciPy's CSR product;
  * fixed-iteration trajectories: per-pass alpha, omega, rho within
    1e-12 + 50 x the running envelope; iterates likewise;
  * converged solves: the iterate after the GPU's pass count within
    max(1e-8, 4 x envelope) of the oracle's iterate after the same count;
    the stop test taken at the GPU's first crossing of (tol ||b||)^2, with
    per-pass estimates tracking the oracle's; true relative residual
    <= 1.1 tol.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from workloads import conv_diff, config_problem, manufactured_rhs, random_sparse, CSR

pytestmark = pytest.mark.gpu

METHODS = [(v, f, p) for v in ("classical", "reordered", "pipelined") for f in ("merged", "basic") for p in ("none", "jacobi")]
# the fused forms (not Improved); their oracle is the merged listing, with
# Jacobi folded into the products
METHODS += [(v, "fused", p) for v in ("classical", "reordered", "pipelined") for p in ("none", "jacobi")]
# Improved BiCGStab (Alg. 3) has no preconditioned form
METHODS += [("improved", f, "none") for f in ("merged", "basic")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_solver(lib, A: CSR, k, variant="classical", formulation="merged", precond="none", precision="fp64"):
    return lib.Solver.from_csr(A, k, variant=variant, formulation=formulation, precond=precond, precision=precision)


def to_np(t):
    return t.detach().cpu().numpy()


# ------------------------------------------------------------------ SpMM ---

@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 8, 13, 16, 32, 64])
def test_spmm_bitwise(lib, k):
    import torch

    say(f"spmm k={k}")
    A = random_sparse(3001, 9, seed=k)
    S = A.to_scipy()
    rng = np.random.default_rng(100 + k)
    X = rng.uniform(-1, 1, (A.n, k))
    s = gpu_solver(lib, A, k)
    Y = to_np(s.spmm(torch.from_numpy(X).cuda()))
    torch.cuda.synchronize()
    assert np.array_equal(Y, S @ X)


@pytest.mark.parametrize("k", [32])
def test_tiled_product_matches_row_order(lib, k):
    """A 3D grid matrix (7-point 24^3, 27-point 16^3 with random values) at
    k = 32 is stored tile by tile for the plain product (its layout
    reported), and that product equals SciPy's CSR product and the row-ordered
    one (BICGSTAB_SPMM_TILE=0 at create) bit for bit; so do a classical merged
    Jacobi solve's pass counts and iterates; after update_values the tiled
    copy carries the new values; a random matrix, and the grid at k = 16, are
    not tiled."""
    import os
    import torch

    from workloads.generators import random_27pt

    say(f"tiled product k={k}")
    rng = np.random.default_rng(40 + k)
    for A, grid in ((conv_diff(24, 3, (1.0, 0.7, 0.3)), (24, 24, 24)), (random_27pt(16, seed=3), (16, 16, 16))):
        X = torch.from_numpy(rng.uniform(-1, 1, (A.n, k))).cuda()
        st = gpu_solver(lib, A, k, precond="jacobi")
        tile, g = st.product_layout()
        assert g == grid and tile == (2, 4, 4), (tile, g)
        os.environ["BICGSTAB_SPMM_TILE"] = "0"
        try:
            sr = gpu_solver(lib, A, k, precond="jacobi")
        finally:
            del os.environ["BICGSTAB_SPMM_TILE"]
        assert sr.product_layout() == ((0, 0, 0), (0, 0, 0))
        Yt = to_np(st.spmm(X))
        Yr = to_np(sr.spmm(X))
        assert np.array_equal(Yt, Yr) and np.array_equal(Yt, A.to_scipy() @ to_np(X))
        b = torch.from_numpy(manufactured_rhs(A, k, seed=7)[0]).cuda()
        xt, it = st.solve(b, tol=1e-8, maxit=500)
        xr, ir = sr.solve(b, tol=1e-8, maxit=500)
        assert np.array_equal(it.iters, ir.iters) and np.array_equal(to_np(xt), to_np(xr))
        # new values through the same array: the tiled copy follows
        A2 = CSR(A.n, A.row_ptr, A.col_idx, A.values * 1.5)
        st.update_values(torch.from_numpy(A2.values).cuda())
        assert np.array_equal(to_np(st.spmm(X)), A2.to_scipy() @ to_np(X))
        st.close()
        sr.close()
    A = random_sparse(4096, 7, seed=1)
    s = gpu_solver(lib, A, k)
    assert s.product_layout() == ((0, 0, 0), (0, 0, 0))
    s.close()
    s = gpu_solver(lib, conv_diff(24, 3, (1.0, 0.7, 0.3)), 16)
    assert s.product_layout() == ((0, 0, 0), (0, 0, 0))
    s.close()


def test_tiled_folded_product_pipelined_fused(lib):
    """The fused Pipelined form with Jacobi runs its plain products on A M^{-1};
    on a 3D grid at k = 32 those read a tile-ordered copy of the folded values.
    Its solve equals the row-ordered one (BICGSTAB_SPMM_TILE=0 at create) bit
    for bit, and the oracle's in the kernels' order on two columns; after
    update_values the folded tile copy carries the new values (the two
    handles still agree, and the oracle on the new matrix)."""
    import os
    import torch

    say("tiled folded product, pipelined fused jacobi k=32")
    A = conv_diff(24, 3, (1.0, 0.7, 0.3))
    k = 32
    b_np = manufactured_rhs(A, k, seed=12)[0]
    b = torch.from_numpy(b_np).cuda()
    st = gpu_solver(lib, A, k, "pipelined", "fused", "jacobi")
    assert st.product_layout() == ((2, 4, 4), (24, 24, 24))
    os.environ["BICGSTAB_SPMM_TILE"] = "0"
    try:
        sr = gpu_solver(lib, A, k, "pipelined", "fused", "jacobi")
    finally:
        del os.environ["BICGSTAB_SPMM_TILE"]
    assert sr.product_layout() == ((0, 0, 0), (0, 0, 0))
    for step, M in ((0, A), (1, CSR(A.n, A.row_ptr, A.col_idx, A.values * np.linspace(0.5, 1.5, A.nnz)))):
        if step:
            for s in (st, sr):
                s.update_values(torch.from_numpy(M.values).cuda())
        xt, it = st.solve(b, tol=1e-8, maxit=500)
        xr, ir = sr.solve(b, tol=1e-8, maxit=500)
        assert np.all(it.status == oracle.CONVERGED)
        assert np.array_equal(it.iters, ir.iters) and np.array_equal(to_np(xt), to_np(xr))
        X = to_np(xt)
        for c in (0, k - 1):
            with oracle_dot(fused_dot(M, k, "pipelined")):
                ref = oracle.solve_column(M.to_scipy(), b_np[:, c], None, "pipelined", "fused", "jacobi", 1e-8, 500)
            assert int(it.iters[c]) == ref.iters and np.array_equal(X[:, c], ref.x), (step, c)
    st.close()
    sr.close()


def test_spmm_and_solve_unaligned_operands(lib):
    """Blocks that start one element past an aligned address (views into a
    larger buffer) take the one-column-per-lane product: the same sums, so
    the product and a whole solve equal those on aligned blocks bit for bit."""
    import torch

    say("spmm unaligned operands")
    A = conv_diff(13, 3, (1.0, 0.7, 0.3))
    k = 6
    n = A.n
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (n, k))
    s = gpu_solver(lib, A, k)
    Y = to_np(s.spmm(torch.from_numpy(X).cuda()))
    assert np.array_equal(Y, A.to_scipy() @ X)
    buf_x = torch.zeros(n * k + 1, dtype=torch.float64, device="cuda")
    buf_y = torch.zeros(n * k + 1, dtype=torch.float64, device="cuda")
    xv = buf_x[1:].view(n, k)
    yv = buf_y[1:].view(n, k)
    assert xv.data_ptr() % 16 == 8 and yv.data_ptr() % 16 == 8
    xv.copy_(torch.from_numpy(X))
    s.spmm(xv, out=yv)
    assert np.array_equal(to_np(yv), Y)
    b, _ = manufactured_rhs(A, k, seed=9)
    x_al, info_al = s.solve(torch.from_numpy(b).cuda(), tol=1e-10, maxit=500)
    bv = buf_y[1:].view(n, k)
    bv.copy_(torch.from_numpy(b))
    xu = buf_x[1:].view(n, k)
    xu.zero_()
    s2 = gpu_solver(lib, A, k)
    x_un, info_un = s2.solve(bv, tol=1e-10, maxit=500, out=xu)
    assert x_un.data_ptr() % 16 == 8
    assert np.array_equal(info_al.iters, info_un.iters)
    assert np.array_equal(to_np(x_al), to_np(x_un))


def test_spmm_long_rows_and_empty_rows(lib):
    """Rows longer than the LDS budget take the split path (different
    summation order: a few ulp); empty rows give zeros."""
    import torch

    say("spmm long rows")
    n = 5000
    rng = np.random.default_rng(7)
    rows = []
    for i in range(n):
        if i in (3, 4000):
            cols = np.sort(rng.choice(n, 4500, replace=False))
        elif i % 97 == 0:
            cols = np.array([], dtype=np.int64)
        else:
            cols = np.sort(rng.choice(n, 5, replace=False))
        rows.append(cols)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(c) for c in rows])
    A = CSR(n, rp.astype(np.int32), np.concatenate(rows).astype(np.int32), rng.uniform(-1, 1, int(rp[-1])))
    S = A.to_scipy()
    for k in (1, 6, 32):
        X = rng.uniform(-1, 1, (n, k))
        s = gpu_solver(lib, A, k)
        Y = to_np(s.spmm(torch.from_numpy(X).cuda()))
        R = S @ X
        scale = (abs(S) @ abs(X)) + 1e-300
        assert np.all(np.abs(Y - R) <= 64 * np.finfo(float).eps * scale)
        short = np.array([len(c) <= 2048 for c in rows])
        assert np.array_equal(Y[short], R[short])


# --------------------------------------------------------- trajectories ---

def _chunked_dot(u, w, chunk=256):
    p = np.multiply(u, w)
    m = (p.size + chunk - 1) // chunk
    q = np.zeros(m * chunk)
    q[: p.size] = p
    return float(q.reshape(m, chunk).sum(axis=1).sum())


DOT_ORDERS = {
    "exact": lambda u, w: __import__("math").fsum(np.multiply(u, w)),
    "reversed": lambda u, w: float(np.sum(np.multiply(u, w)[::-1])),
    "chunked": _chunked_dot,
}


def oracle_with_dots(order, *args, **kw):
    """The oracle with its dot products summed in another order (exactly
    rounded, reversed pairwise, or per-256-chunk like a GPU tree): the spread
    between such runs and the plain oracle is how far summation order alone
    moves a trajectory, the envelope the GPU (one more order) must stay in."""
    import oracle.bicgstab as ob

    saved = ob.dot
    ob.dot = DOT_ORDERS[order]
    try:
        return oracle.solve(*args, **kw)
    finally:
        ob.dot = saved


def oracle_with_exact_dots(*args, **kw):
    return oracle_with_dots("exact", *args, **kw)


@pytest.mark.parametrize("variant,formulation,precond", METHODS)
@pytest.mark.parametrize("k", [1, 5])
def test_trajectory_fixed_iterations(lib, variant, formulation, precond, k):
    """20 passes with the stop test off: per-pass alpha, omega, rho and the
    final iterate match the oracle within 1e-12 plus 50x the summation-order
    envelope (which reaches ~1e-9 by pass 20 as the residual falls)."""
    import torch

    say(f"trajectory {variant}/{formulation}/{precond} k={k}")
    A = conv_diff(17, 3, (1.0, 0.7, 0.3))
    b, _ = manufactured_rhs(A, k, seed=21)
    nit = 20
    s = gpu_solver(lib, A, k, variant, formulation, precond)
    x, info = s.solve(torch.from_numpy(b).cuda(), tol=0.0, maxit=nit)
    hist = s.history()
    kw = dict(variant=variant, formulation=formulation, precond=precond, tol=0.0, maxit=nit, trace=True)
    ref = oracle.solve(A.to_scipy(), b, **kw)
    alts = [oracle_with_dots(o, A.to_scipy(), b, **kw) for o in DOT_ORDERS]
    assert np.all(info.status == oracle.MAXIT) and np.all(info.iters == nit)
    X = to_np(x)
    keys = ((0, "alpha"), (1, "omega"), (2, "rho"))
    for c in range(k):
        nref = np.linalg.norm(ref.x[:, c])
        spread = max(np.linalg.norm(a.x[:, c] - ref.x[:, c]) / nref for a in alts)
        err = np.linalg.norm(X[:, c] - ref.x[:, c]) / nref
        assert err < 1e-12 + 20 * spread, (c, err, spread)
        tr = ref.traces[c]
        env = 0.0  # running maximum of the relative summation-order spread
        for j in range(nit):
            env = max([env] + [abs(a.traces[c][j][key] - tr[j][key]) / abs(tr[j][key]) for a in alts for _, key in keys])
            for idx, key in keys:
                g, o = hist[j, c, idx], tr[j][key]
                assert abs(g - o) <= (1e-12 + 20 * env) * abs(o), (c, j, key, g, o, env)


# --------------------------------------------------------------- solves ---

def _check_solve(lib, A, b, variant, formulation, precond, tol, maxit=3000, x0=None):
    """Converged GPU solve vs the oracle, per column c with GPU pass count j:
      * converged, with true relative residual <= 1.1 tol;
      * the iterate after j passes equals the oracle's iterate after j passes
        (stop test off) within max(1e-8, 4 x the summation-order spread
        between the oracle and three reorderings of its dot products,
        pooled over the columns);
      * the stop test: the GPU stopped at the first pass where its own
        estimate fell below (tol ||b||)^2, and its per-pass estimates track the
        oracle's (within a factor 10) while those are above 1e-6 of the first
        and before the oracle's first tenfold jump.
        (The stopping pass itself is not compared: BiCGStab's estimate
        plateaus near the threshold, so two oracle runs that differ only in
        dot-product order stop up to 13 passes apart on the 64 x 64 case.)
    """
    import torch

    s = gpu_solver(lib, A, b.shape[1], variant, formulation, precond)
    x, info = s.solve(torch.from_numpy(b).cuda(), None if x0 is None else torch.from_numpy(x0).cuda(), tol=tol,
                      maxit=maxit)
    hist = s.history()
    S = A.to_scipy()
    X = to_np(x)
    assert np.all(info.status == oracle.CONVERGED), info.status
    assert np.all(info.relres_true <= 1.1 * tol), info.relres_true
    errs, spreads, refs = [], [], []
    for c in range(b.shape[1]):
        j = int(info.iters[c])
        bc = b[:, c]
        x0c = None if x0 is None else x0[:, c]
        kw = dict(variant=variant, formulation=formulation, precond=precond, tol=0.0, maxit=j, trace=True)
        ref = oracle.solve(S, bc, x0c, **kw)
        nref = np.linalg.norm(ref.x[:, 0])
        spreads.append(max(np.linalg.norm(oracle_with_dots(o, S, bc, x0c, **kw).x[:, 0] - ref.x[:, 0]) / nref
                           for o in DOT_ORDERS))
        errs.append(np.linalg.norm(X[:, c] - ref.x[:, 0]) / nref)
        refs.append(ref)
    # the envelope is pooled over the columns (same matrix, similar pass
    # counts): a single column's three reorderings can agree by chance
    envelope = max(spreads)
    assert max(errs) <= max(1e-8, 4 * envelope), (errs, spreads)
    for c in range(b.shape[1]):
        j = int(info.iters[c])
        bc = b[:, c]
        eps2 = tol * tol * float(bc @ bc)
        ref = refs[c]
        if j > 0:
            eg = hist[:j, c, 3]
            eo = np.array([t["est"] for t in ref.traces[0]])
            assert eg[j - 1] < eps2 * (1 + 1e-12) and np.all(eg[: j - 1] >= eps2 * (1 - 1e-12)), (c, j)
            # while the oracle's estimate is above 1e-6 of the first, and
            # before its first jump by more than 10x: BiCGStab's residual is
            # not monotone, and where a spike appears depends on rounding (a
            # rounding-level change such as the fused form's folded Jacobi
            # products moves it), after which two runs no longer follow one path
            jump = np.nonzero(eo[1:] > 10 * eo[:-1])[0]
            live = eo > 1e-6 * eo[0]
            if jump.size:
                live[jump[0] + 1:] = False
            ratio = eg[live] / eo[live]
            assert np.all((ratio > 0.1) & (ratio < 10)), (c, ratio)
    # the library's own true residual agrees with one recomputed on the host
    rt = np.linalg.norm(b - A.to_scipy() @ X, axis=0) / np.linalg.norm(b, axis=0)
    assert np.allclose(info.relres_true, rt, rtol=1e-6, atol=1e-16)
    return info, ref


@pytest.mark.parametrize("variant,formulation,precond", METHODS)
def test_solve_small_2d(lib, variant, formulation, precond):
    """The 2D 5-point convection-diffusion recipe at 64 x 64, one RHS,
    tol 1e-10."""
    say(f"solve 2d {variant}/{formulation}/{precond}")
    cfg = config_problem(0, seed=0)
    _check_solve(lib, cfg["A"], cfg["b"], variant, formulation, precond, cfg["tol"])


@pytest.mark.parametrize("variant,formulation,precond", METHODS)
@pytest.mark.parametrize("k", [3, 8])
def test_solve_3d_multi_rhs(lib, variant, formulation, precond, k):
    """The 3D 7-point recipe at 21^3 (several row blocks and a ragged tail),
    Jacobi or not, tol 1e-8."""
    say(f"solve 3d {variant}/{formulation}/{precond} k={k}")
    cfg = config_problem(1, seed=1, k=k, scale=21)
    _check_solve(lib, cfg["A"], cfg["b"], variant, formulation, precond, cfg["tol"])


def test_solve_random_sparse(lib):
    say("solve random sparse")
    A = random_sparse(20000, 15, seed=4)
    b, _ = manufactured_rhs(A, 4, seed=5)
    for m in METHODS:
        _check_solve(lib, A, b, *m, tol=1e-10)


def test_solve_k32_and_k64(lib):
    say("solve k=32, k=64")
    A = conv_diff(12, 3, (1.0, 0.7, 0.3))
    for k in (32, 64):
        b, _ = manufactured_rhs(A, k, seed=k)
        _check_solve(lib, A, b, "classical", "merged", "jacobi", 1e-9)
        _check_solve(lib, A, b, "pipelined", "merged", "none", 1e-9)


# ---------------------------------------------------------------- edges ---

@pytest.mark.parametrize("variant,formulation,precond", METHODS)
def test_edge_columns(lib, variant, formulation, precond):
    """Zero column, NaN column, maxit = 1, exact initial guess, identical
    columns: same statuses and counts as the oracle."""
    import torch

    say(f"edges {variant}/{formulation}/{precond}")
    A = conv_diff(6, 2, (1.0, 0.5))
    S = A.to_scipy()
    n = A.n
    rng = np.random.default_rng(15)
    xs = rng.uniform(-1, 1, n)
    B = np.stack([np.zeros(n), S @ xs, S @ xs, S @ xs, S @ xs], axis=1)
    B[3, 1] = np.nan
    X0 = np.zeros_like(B)
    X0[:, 3] = xs
    X0[:, 0] = 1.0
    s = gpu_solver(lib, A, 5, variant, formulation, precond)
    x, info = s.solve(torch.from_numpy(B).cuda(), torch.from_numpy(X0).cuda(), tol=1e-10, maxit=1)
    ref = oracle.solve(S, B, X0, variant, formulation, precond, 1e-10, 1)
    assert list(info.status) == list(ref.status)
    assert list(info.iters) == list(ref.iters)
    X = to_np(x)
    assert np.all(X[:, 0] == 0) and np.array_equal(X[:, 3], xs)
    assert np.array_equal(X[:, 2], X[:, 4])  # identical columns, identical results


def test_breakdown_and_scaled_identity(lib):
    import torch

    say("breakdown / cI")
    skew = CSR(2, np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, -1.0]))
    b = np.array([[1.0], [2.0]])
    for v, f, p in METHODS:
        if p == "jacobi":
            continue
        s = gpu_solver(lib, skew, 1, v, f, p)
        x, info = s.solve(torch.from_numpy(b).cuda(), tol=1e-10, maxit=10)
        assert info.status[0] == oracle.BREAKDOWN
        assert info.iters[0] == (0 if v == "pipelined" else 1)
    n = 33
    for c in (2.0, 3.0):
        A = CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.full(n, c))
        b = np.random.default_rng(3).uniform(-1, 1, (n, 2))
        for v, f, p in METHODS:
            s = gpu_solver(lib, A, 2, v, f, p)
            x, info = s.solve(torch.from_numpy(b).cuda(), tol=1e-12, maxit=10)
            assert np.all(info.status == 0) and np.all(info.iters == 1)
            assert np.allclose(to_np(x), b / c, rtol=1e-15, atol=0)


def test_jacobi_zero_diagonal_is_error(lib):
    import torch

    say("jacobi zero diagonal")
    skew = CSR(2, np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, -1.0]))
    s = gpu_solver(lib, skew, 1, "classical", "merged", "jacobi")
    with pytest.raises(lib.BicgstabError):
        s.solve(torch.ones(2, 1, dtype=torch.float64).cuda())


def test_empty_system(lib):
    import torch

    say("n = 0")
    A = CSR(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    s = gpu_solver(lib, A, 3)
    x, info = s.solve(torch.zeros(0, 3, dtype=torch.float64).cuda(), tol=1e-8, maxit=10)
    assert x.shape == (0, 3) and np.all(info.status == 0) and np.all(info.iters == 0)


def test_bad_column_index_rejected(lib):
    say("bad column index")
    A = CSR(3, np.array([0, 1, 2, 3], np.int32), np.array([0, 5, 2], np.int32), np.ones(3))
    with pytest.raises(lib.BicgstabError):
        gpu_solver(lib, A, 1)


@pytest.mark.parametrize("variant,formulation", [("pipelined", "merged"), ("classical", "fused")])
def test_deterministic_and_graph_equals_direct(lib, monkeypatch, variant, formulation):
    import torch

    say(f"determinism {variant} {formulation}")
    cfg = config_problem(1, seed=3, k=4, scale=16)
    b = torch.from_numpy(cfg["b"]).cuda()
    s = gpu_solver(lib, cfg["A"], 4, variant, formulation, "jacobi")
    x1, i1 = s.solve(b, tol=1e-8, maxit=500)
    x2, i2 = s.solve(b, tol=1e-8, maxit=500)
    assert torch.equal(x1, x2) and np.array_equal(i1.iters, i2.iters)
    monkeypatch.setenv("BICGSTAB_GRAPH", "0")
    monkeypatch.setenv("BICGSTAB_CHUNK", "3")
    s2 = gpu_solver(lib, cfg["A"], 4, variant, formulation, "jacobi")
    x3, i3 = s2.solve(b, tol=1e-8, maxit=500)
    assert torch.equal(x1, x3) and np.array_equal(i1.iters, i3.iters)


def test_fused_equals_merged_up_to_dot_order(lib):
    """The fused classical form computes the merged form's statements (with
    Jacobi, its products read A M^{-1} instead of applying M^{-1} first, a
    rounding-level change): 20 fixed passes of both forms agree within the
    summation-order envelope of the oracle."""
    import torch

    say("fused vs merged")
    A = conv_diff(15, 3, (1.0, -0.4, 0.6))
    b, _ = manufactured_rhs(A, 6, seed=31)
    for precond in ("none", "jacobi"):
        xs = {}
        for f in ("merged", "fused"):
            s = gpu_solver(lib, A, 6, "classical", f, precond)
            x, info = s.solve(torch.from_numpy(b).cuda(), tol=0.0, maxit=20)
            assert np.all(info.iters == 20)
            xs[f] = to_np(x)
        kw = dict(variant="classical", formulation="merged", precond=precond, tol=0.0, maxit=20)
        ref = oracle.solve(A.to_scipy(), b, **kw)
        alts = [oracle_with_dots(o, A.to_scipy(), b, **kw) for o in DOT_ORDERS]
        for c in range(6):
            nref = np.linalg.norm(ref.x[:, c])
            spread = max(np.linalg.norm(a.x[:, c] - ref.x[:, c]) / nref for a in alts)
            d = np.linalg.norm(xs["fused"][:, c] - xs["merged"][:, c]) / nref
            assert d <= 1e-12 + 40 * spread, (precond, c, d, spread)


# ----------------------------------------------------------- bitwise ---

from kernel_order import group_dot, oracle_dot, scheduled_dot, spmm_epilogue_dot, tile_order  # noqa: E402

BITWISE = [m for m in METHODS if m[1] != "fused"]


@pytest.mark.parametrize("variant,formulation,precond", BITWISE)
@pytest.mark.parametrize("k", [1, 5])
def test_bitwise_fixed_passes(lib, variant, formulation, precond, k):
    """20 passes with the stop test off: every iterate and every per-pass
    alpha, omega, rho and stop estimate equal the oracle's in the kernels'
    summation order."""
    import torch

    say(f"bitwise passes {variant}/{formulation}/{precond} k={k}")
    A = conv_diff(17, 3, (1.0, 0.7, 0.3))
    b, _ = manufactured_rhs(A, k, seed=21)
    s = gpu_solver(lib, A, k, variant, formulation, precond)
    x, info = s.solve(torch.from_numpy(b).cuda(), tol=0.0, maxit=20)
    hist = s.history()
    with oracle_dot(group_dot(A.n, k)):
        ref = oracle.solve(A.to_scipy(), b, variant=variant, formulation=formulation, precond=precond, tol=0.0,
                           maxit=20, trace=True)
    X = to_np(x)
    assert np.array_equal(info.iters, ref.iters) and np.array_equal(info.status, ref.status)
    for c in range(k):
        assert np.array_equal(X[:, c], ref.x[:, c]), (c, np.abs(X[:, c] - ref.x[:, c]).max())
        for j, t in enumerate(ref.traces[c]):
            got = tuple(hist[j, c, :])
            want = (t["alpha"], t["omega"], t["rho"], t["est"])
            assert got == want, (c, j, got, want)


@pytest.mark.parametrize("variant,formulation,precond", BITWISE)
def test_bitwise_converged(lib, variant, formulation, precond):
    """Solves to tolerance on the 2D recipe (64 x 64, tol 1e-10) and the 3D
    recipe (16^3, k = 4, tol 1e-8): pass counts, statuses and solutions equal
    the oracle's in the kernels' summation order (so also within any pass
    count margin and relative error bar)."""
    import torch

    for cfg in (config_problem(0, seed=2, k=2), config_problem(1, seed=3, k=4, scale=16)):
        A, b, tol = cfg["A"], cfg["b"], cfg["tol"]
        say(f"bitwise converged {variant}/{formulation}/{precond} n={A.n} k={b.shape[1]}")
        s = gpu_solver(lib, A, b.shape[1], variant, formulation, precond)
        x, info = s.solve(torch.from_numpy(b).cuda(), tol=tol, maxit=3000)
        with oracle_dot(group_dot(A.n, b.shape[1])):
            ref = oracle.solve(A.to_scipy(), b, variant=variant, formulation=formulation, precond=precond, tol=tol,
                               maxit=3000)
        assert np.array_equal(info.status, ref.status), (info.status, ref.status)
        assert np.array_equal(info.iters, ref.iters), (info.iters, ref.iters)
        assert np.array_equal(to_np(x), ref.x)


def fused_dot(A, k, variant="classical", solver=None):
    """A fused form's dot sequence: (r, r), (b, b) from the start pass, then
    per pass: classical, delta from the first product's epilogue, phi, psi,
    theta from the second's and rho' from a vector pass; Reordered, delta from
    the first product's epilogue and theta, phi, psi, eta from a vector
    pass (from k = 4 on, from the second product's epilogue). solver: the handle whose
    layout the products follow (a tile-ordered copy of A makes the epilogues
    add its rows in the stored order)."""
    g = group_dot(A.n, k)
    perm = None
    if solver is not None:
        tile, grid = solver.product_layout()
        if tile[0] > 0:
            perm = tile_order(grid, tile)
    e = spmm_epilogue_dot(A.row_ptr, k, perm=perm)
    if variant == "pipelined":  # no product epilogue dots: every dot from a vector pass
        return g
    if variant == "reordered":
        return scheduled_dot([g, g], [e, e, e, e, e] if k >= 4 else [e, g, g, g, g])
    return scheduled_dot([g, g], [e, e, e, e, g])


@pytest.mark.parametrize("variant", ["classical", "reordered", "pipelined"])
@pytest.mark.parametrize("precond", ["none", "jacobi"])
@pytest.mark.parametrize("k", [5, 6])
def test_bitwise_fused(lib, variant, precond, k):
    """The fused forms, 20 fixed passes and a converged solve, per
    column (each column's oracle run gets its own dot schedule): iterates,
    pass counts and statuses equal the oracle's in the kernels' order. Odd k
    runs the product one column per lane, even k two (k = 6: a padded lane
    pair)."""
    import torch

    A = conv_diff(17, 3, (1.0, 0.7, 0.3))
    b, _ = manufactured_rhs(A, k, seed=22)
    S = A.to_scipy()
    for tol, maxit in ((0.0, 20), (1e-10, 3000)):
        say(f"bitwise fused {variant} {precond} k={k} tol={tol}")
        s = gpu_solver(lib, A, k, variant, "fused", precond)
        x, info = s.solve(torch.from_numpy(b).cuda(), tol=tol, maxit=maxit)
        X = to_np(x)
        for c in range(k):
            with oracle_dot(fused_dot(A, k, variant, s)):
                ref = oracle.solve_column(S, b[:, c], None, variant, "fused", precond, tol, maxit)
            assert (int(info.iters[c]), int(info.status[c])) == (ref.iters, ref.status), (c, info.iters[c], ref.iters)
            assert np.array_equal(X[:, c], ref.x), (c, np.abs(X[:, c] - ref.x).max())


@pytest.mark.parametrize("variant", ["classical", "reordered", "pipelined"])
def test_bitwise_fused_k64_multichunk(lib, variant):
    """k = 64 (the largest), Jacobi, on 52^3 rows: the products' epilogue
    partials of up to 3 x 64 pairs are summed in runs of about 34 row blocks,
    more than one LDS chunk (32 blocks at 192 pairs) each. Three fused passes
    equal the oracle's in the kernels' order on the first and last column."""
    import torch

    say(f"bitwise fused k=64 multichunk {variant}")
    A = conv_diff(52, 3, (1.0, 0.7, 0.3))
    k = 64
    b, _ = manufactured_rhs(A, k, seed=23)
    S = A.to_scipy()
    s = gpu_solver(lib, A, k, variant, "fused", "jacobi")
    x, info = s.solve(torch.from_numpy(b).cuda(), tol=0.0, maxit=3)
    X = to_np(x)
    for c in (0, k - 1):
        with oracle_dot(fused_dot(A, k, variant, s)):
            ref = oracle.solve_column(S, b[:, c], None, variant, "fused", "jacobi", 0.0, 3)
        assert np.array_equal(X[:, c], ref.x), (c, np.abs(X[:, c] - ref.x).max())


@pytest.mark.parametrize("formulation", ["merged", "basic", "fused"])
def test_reordered_restart_bitwise(lib, formulation):
    """Reordered BiCGStab with Jacobi at k = 32 on 24^3 rows, to tol 1e-8:
    the restart test of the rho recurrence fires (the oracle's trace says
    where), and the library takes the same restarts: pass counts, statuses,
    solutions and every pass's alpha, omega, rho and stop estimate equal the
    oracle's in the kernels' summation order."""
    import torch

    say(f"reordered restart bitwise {formulation}")
    A = conv_diff(24, 3, (1.0, 0.7, 0.3))
    k = 32
    b, _ = manufactured_rhs(A, k, seed=0)
    S = A.to_scipy()
    s = gpu_solver(lib, A, k, "reordered", formulation, "jacobi")
    x, info = s.solve(torch.from_numpy(b).cuda(), tol=1e-8, maxit=500)
    hist = s.history()
    X = to_np(x)
    restarts = 0
    for c in range(k):
        tr = []
        with oracle_dot(fused_dot(A, k, "reordered", s) if formulation == "fused" else group_dot(A.n, k)):
            ref = oracle.solve_column(S, b[:, c], None, "reordered", formulation, "jacobi", 1e-8, 500, trace=tr)
        restarts += sum(bool(t["restart"]) for t in tr)
        assert (int(info.iters[c]), int(info.status[c])) == (ref.iters, ref.status), (c, info.iters[c], ref.iters)
        assert np.array_equal(X[:, c], ref.x), (c, np.abs(X[:, c] - ref.x).max())
        for j, t in enumerate(tr):
            assert tuple(hist[j, c, :]) == (t["alpha"], t["omega"], t["rho"], t["est"]), (c, j)
    assert restarts > 0
    assert np.all(info.status == 0)


def test_reordered_restart_full_size(lib):
    """The column that ran to the pass limit before the restart test existed
    (128^3 7-point, Jacobi, k = 32, fused Reordered form, column 19): 36
    passes, with the restart the oracle takes at pass 31, equal bit for bit
    (iterate and per-pass scalars) to the oracle in the kernels' order."""
    import torch

    say("reordered restart full size 128^3 k=32 fused, 36 passes")
    cfg = config_problem(1, seed=0, k=32)
    A, b = cfg["A"], cfg["b"]
    s = gpu_solver(lib, A, 32, "reordered", "fused", "jacobi")
    x, info = s.solve(torch.from_numpy(b).cuda(), tol=1e-8, maxit=36)
    hist = s.history()
    c = 19
    tr = []
    with oracle_dot(fused_dot(A, 32, "reordered", s)):
        ref = oracle.solve_column(A.to_scipy(), b[:, c], None, "reordered", "fused", "jacobi", 1e-8, 36, trace=tr)
    assert any(t["restart"] for t in tr)
    assert np.array_equal(to_np(x)[:, c], ref.x)
    for j, t in enumerate(tr):
        assert tuple(hist[j, c, :]) == (t["alpha"], t["omega"], t["rho"], t["est"]), j


@pytest.mark.parametrize("variant,formulation,precond", [("classical", "merged", "jacobi"), ("classical", "merged", "none"),
                                                         ("classical", "basic", "jacobi"), ("classical", "fused", "jacobi"),
                                                         ("reordered", "merged", "none"), ("reordered", "fused", "none")])
def test_pending_scalar_step_changes_nothing(lib, monkeypatch, variant, formulation, precond):
    """At small k an alpha or omega reduction hands its scalar step to the
    next pass (no one-workgroup finalize kernel): solutions, pass counts,
    statuses and per-pass scalars equal those of the same solve with every
    step in its own finalize kernel (BICGSTAB_FOLD_MAX=0), bit for bit, with
    fewer kernel launches per iteration."""
    import torch

    say(f"pending scalar step {variant}/{formulation}/{precond}")
    A = conv_diff(19, 3, (1.0, 0.7, 0.3))
    b, _ = manufactured_rhs(A, 3, seed=41)
    bt = torch.from_numpy(b).cuda()
    res = {}
    for fold in ("8192", "0"):
        monkeypatch.setenv("BICGSTAB_FOLD_MAX", fold)
        s = gpu_solver(lib, A, 3, variant, formulation, precond)
        x, info = s.solve(bt, tol=1e-9, maxit=2000)
        res[fold] = (to_np(x), info.iters.copy(), info.status.copy(), s.history(), s.stats())
        s.close()
    (x1, i1, s1, h1, st1), (x0, i0, s0, h0, st0) = res["8192"], res["0"]
    assert np.array_equal(i1, i0) and np.array_equal(s1, s0) and np.all(s1 == 0)
    assert np.array_equal(x1, x0)
    for c in range(3):  # the passes each column ran (the rest of the history is not written)
        assert np.array_equal(h1[: i1[c], c], h0[: i0[c], c]), c
    assert st1["iterations_enqueued"] == st0["iterations_enqueued"]
    assert st1["launches"] < st0["launches"], (st1, st0)


# ---------------------------------------------------- full-size checks ---

def test_full_size_cfg1_sampled(lib):
    """The 128^3 7-point Jacobi workload at k = 32 (the benchmark's launch
    configuration): SpMM rows sampled against the oracle's product, three
    passes of every merged method and of the fused form bit for bit against
    the oracle (kernel summation order) on columns 0 and 31, and a converged
    classical solve checked by its recomputed residual and the manufactured
    solution."""
    import torch

    say("full size 128^3 k=32")
    cfg = config_problem(1, seed=0, k=32)
    A, b, xs = cfg["A"], cfg["b"], cfg["x_star"]
    S = A.to_scipy()
    bt = torch.from_numpy(b).cuda()
    s = gpu_solver(lib, A, 32, "classical", "merged", "jacobi")
    Y = to_np(s.spmm(bt))
    rows = np.random.default_rng(0).choice(A.n, 2000, replace=False)
    assert np.array_equal(Y[rows], S[rows] @ b)
    for v, f in (("classical", "merged"), ("reordered", "merged"), ("pipelined", "merged"), ("classical", "fused"),
                 ("reordered", "fused"), ("pipelined", "fused")):
        say(f"  3 passes {v} {f} (bitwise)")
        s3 = gpu_solver(lib, A, 32, v, f, "jacobi")
        x, info = s3.solve(bt, tol=0.0, maxit=3)
        X = to_np(x)
        for c in (0, 31):
            with oracle_dot(fused_dot(A, 32, v, s3) if f == "fused" else group_dot(A.n, 32)):
                ref = oracle.solve_column(S, b[:, c], None, v, f, "jacobi", 0.0, 3)
            assert np.array_equal(X[:, c], ref.x), (v, f, c)
        del s3
    say("  converged solve")
    x, info = s.solve(bt, tol=1e-8, maxit=2000)
    X = to_np(x)
    assert np.all(info.status == 0)
    rt = np.linalg.norm(b - S @ X, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(rt <= 1.1e-8) and np.allclose(rt, info.relres_true, rtol=1e-6)
    assert np.all(np.linalg.norm(X - xs, axis=0) / np.linalg.norm(xs, axis=0) < 1e-4)


def test_full_size_random_sparse_sampled(lib):
    """The random sparse matrix of the benchmark (n = 2^21, 15 random columns
    per row) at k = 32: SpMM rows sampled against the oracle's product, three
    classical merged Jacobi passes bit for bit against the oracle on columns
    0 and 31, and a converged solve checked by its recomputed residual."""
    import torch

    say("full size random sparse 2^21 k=32")
    A = random_sparse(2**21, 15, seed=0)
    b, xs = manufactured_rhs(A, 32, seed=0)
    S = A.to_scipy()
    bt = torch.from_numpy(b).cuda()
    s = gpu_solver(lib, A, 32, "classical", "merged", "jacobi")
    Y = to_np(s.spmm(bt))
    rows = np.random.default_rng(1).choice(A.n, 2000, replace=False)
    assert np.array_equal(Y[rows], S[rows] @ b)
    say("  3 passes (bitwise)")
    x, _ = s.solve(bt, tol=0.0, maxit=3)
    X = to_np(x)
    for c in (0, 31):
        with oracle_dot(group_dot(A.n, 32)):
            ref = oracle.solve_column(S, b[:, c], None, "classical", "merged", "jacobi", 0.0, 3)
        assert np.array_equal(X[:, c], ref.x), c
    say("  converged solve")
    x, info = s.solve(bt, tol=1e-8, maxit=500)
    X = to_np(x)
    assert np.all(info.status == 0)
    rt = np.linalg.norm(b - S @ X, axis=0) / np.linalg.norm(b, axis=0)
    assert np.all(rt <= 1.1e-8) and np.allclose(rt, info.relres_true, rtol=1e-6)
    assert np.all(np.linalg.norm(X - xs, axis=0) / np.linalg.norm(xs, axis=0) < 1e-5)


# ------------------------------------------------------------ Table 1 ---

def test_table1_updates_gpu(lib):
    """The three runs of Table 1 on the GPU against the updates in NumPy, bit
    for bit: run 1 (three passes) and run 3 (one pass) give the same vectors,
    run 2 the first two updates; odd lengths take the one-element tail."""
    import torch

    say("table 1 updates")
    rng = np.random.default_rng(9)
    for n in (1, 1001, 2**20 + 3):
        x, y0, z0 = (rng.uniform(-1, 1, n) for _ in range(3))
        a, b, c = 0.3, -1.7, 2.5
        xt = torch.from_numpy(x).cuda()
        for run in (1, 2, 3):
            yt, zt = torch.from_numpy(y0).cuda(), torch.from_numpy(z0).cuda()
            lib.axpby_tab1(run, xt, yt, zt, a, b, c)
            torch.cuda.synchronize()
            ry, rz = y0.copy(), z0.copy()
            ry = a * x + b * ry
            rz = b * x + a * rz
            if run != 2:
                rz = b * ry + c * rz
            assert np.array_equal(to_np(yt), ry) and np.array_equal(to_np(zt), rz), (n, run)
    e = torch.zeros(0, dtype=torch.float64, device="cuda")
    lib.axpby_tab1(3, e, e.clone(), e.clone(), 1.0, 1.0, 1.0)
    with pytest.raises(lib.BicgstabError):
        lib.axpby_tab1(4, xt, xt.clone(), xt.clone(), 1.0, 1.0, 1.0)


# ------------------------------------------------------- property test ---

def test_random_systems_property_gpu(lib):
    """Property: on random nonsymmetric systems with a dominant diagonal
    (n 1..3000, k 1..9, every method, form and preconditioner, fixed passes
    or a converged solve), the GPU equals the oracle run in the kernels'
    summation order bit for bit."""
    import torch
    from hypothesis import HealthCheck, given, settings
    from hypothesis import strategies as st

    def system(seed, n, k):
        rng = np.random.default_rng(seed)
        rows, vals = [], []
        for i in range(n):
            cols = np.unique(np.concatenate(([i], rng.choice(n, size=min(n, 4), replace=False))))
            v = rng.uniform(-1, 1, cols.size)
            v[cols == i] = 0.0
            v[cols == i] = 1.5 * np.abs(v).sum() + 1.0
            rows.append(cols)
            vals.append(v)
        rp = np.zeros(n + 1, np.int32)
        rp[1:] = np.cumsum([c.size for c in rows])
        return CSR(n, rp, np.concatenate(rows).astype(np.int32), np.concatenate(vals)), rng.uniform(-1, 1, (n, k))

    @settings(max_examples=30, deadline=None, suppress_health_check=list(HealthCheck))
    @given(seed=st.integers(0, 10**6), n=st.integers(1, 3000), k=st.integers(1, 9), method=st.sampled_from(METHODS),
           tol=st.sampled_from([0.0, 1e-9]))
    def check(seed, n, k, method, tol):
        v, f, p = method
        A, b = system(seed, n, k)
        maxit = 10 if tol == 0.0 else 400
        say(f"property n={n} k={k} {v}/{f}/{p} tol={tol}")
        s = gpu_solver(lib, A, k, v, f, p)
        x, info = s.solve(torch.from_numpy(b).cuda(), tol=tol, maxit=maxit)
        X = to_np(x)
        if f == "fused":
            # each column's oracle run gets the fused plan's dot schedule
            S = A.to_scipy()
            for c in range(k):
                with oracle_dot(fused_dot(A, k, v, s)):
                    ref = oracle.solve_column(S, b[:, c], None, v, f, p, tol, maxit)
                assert (int(info.iters[c]), int(info.status[c])) == (ref.iters, ref.status), c
                assert np.array_equal(X[:, c], ref.x, equal_nan=True), c
            return
        with oracle_dot(group_dot(A.n, k)):
            ref = oracle.solve(A.to_scipy(), b, variant=v, formulation=f, precond=p, tol=tol, maxit=maxit)
        assert np.array_equal(info.iters, ref.iters) and np.array_equal(info.status, ref.status)
        assert np.array_equal(X, ref.x, equal_nan=True)

    check()
