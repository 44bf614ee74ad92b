"""GPU tests of the batched tier (many independent systems in one persistent
launch) against an oracle loop over the systems.

The batched kernel forms every sparse product and vector update in the
oracle's order without contraction, and sums each dot product in a fixed
order that depends only on the system's size, k, its workgroup share and the
workgroup size: per thread over its rows (a stride of block / kp rows through
the workgroup's contiguous row chunk), a pairwise tree over the row slots of a
wave, the waves in index order, then the workgroups in index order. The
tests run the oracle with its dot product summed in that order
(`kernel_order.batched_dot`), which makes the whole solve reproducible bit for bit:
pass counts, statuses and iterates must be identical. The same runs with the
oracle's own dot products stay within the summation-order envelope (checked
in the single-system tests).
"""
import sys

import numpy as np
import pytest

import oracle
from kernel_order import batched_dot, oracle_dot
from workloads import CSR, batched_systems, config_problem, conv_diff, manufactured_rhs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_kernel_order(A, k, nw, block, *args, **kw):
    with oracle_dot(batched_dot(A.n, k, nw, block)):
        return oracle.solve(A.to_scipy(), *args, **kw)


# the oracle of the batched kernel: Alg. 2, or with Jacobi Alg. 5 with M^{-1}
# folded into the products (the single-system path's fused classical form)
METHOD = {"none": {}, "jacobi": {"variant": "classical", "formulation": "fused", "precond": "jacobi"}}


def _batch(nsys, seed, nmin=200, nmax=5000):
    systems = batched_systems(nsys, seed, nmin=nmin, nmax=nmax)
    rhs = [manufactured_rhs(A, k, seed * 1000 + s)[0] for s, (A, k) in enumerate(systems)]
    return systems, rhs


def _gpu_solve(lib, systems, rhs, tol, maxit, x0s=None, solver=None):
    import torch

    bs = lib.BatchedSolver(systems) if solver is None else solver
    xs, infos = bs.solve([torch.from_numpy(b).cuda() for b in rhs],
                         None if x0s is None else [torch.from_numpy(x).cuda() for x in x0s], tol=tol, maxit=maxit)
    return bs, [x.cpu().numpy() for x in xs], infos


def _check_bitwise(bs, systems, rhs, X, infos, tol, maxit, x0s=None, which=None, precond="none"):
    """Per system: the oracle in the kernel's summation order gives the same
    pass counts, statuses and iterates, bit for bit; the library's true
    residual equals one recomputed on the host."""
    cfg = bs.config()
    block, wg = cfg.block, cfg.workgroups
    for s in (range(len(systems)) if which is None else which):
        A, k = systems[s]
        b = rhs[s]
        ref = oracle_kernel_order(A, k, int(wg[s]), block, b, None if x0s is None else x0s[s], tol=tol, maxit=maxit,
                                  **METHOD[precond])
        info = infos[s]
        assert np.array_equal(info.status, ref.status), (s, info.status, ref.status)
        assert np.array_equal(info.iters, ref.iters), (s, info.iters, ref.iters)
        assert np.array_equal(X[s], ref.x), (s, np.abs(X[s] - ref.x).max())
        nb = np.linalg.norm(b, axis=0)
        rt = np.where(nb > 0, np.linalg.norm(b - A.to_scipy() @ X[s], axis=0) / np.where(nb > 0, nb, 1), 0.0)
        assert np.allclose(info.relres_true, rt, rtol=1e-6, atol=1e-300), (s, info.relres_true, rt)


def test_batched_fixed_passes_bitwise(lib):
    """16 systems (2D 5-point and 3D 7-point, n in [200, 5000], k in 1..8),
    12 passes with the stop test off."""
    systems, rhs = _batch(16, seed=1)
    say(f"batched fixed passes: {[(A.n, k) for A, k in systems]}")
    bs, X, infos = _gpu_solve(lib, systems, rhs, tol=0.0, maxit=12)
    for info in infos:
        assert np.all(info.status == oracle.MAXIT) and np.all(info.iters == 12)
    _check_bitwise(bs, systems, rhs, X, infos, 0.0, 12)


def test_batched_converged_bitwise(lib):
    """16 systems to tol 1e-8 with the starting configuration: every column
    converges with a true residual <= 1.1 tol, bit for bit the oracle's."""
    systems, rhs = _batch(16, seed=2)
    say(f"batched converged: {[(A.n, k) for A, k in systems]}")
    bs, X, infos = _gpu_solve(lib, systems, rhs, tol=1e-8, maxit=3000)
    say(f"  passes {[int(i.iters.max()) for i in infos]}")
    for info in infos:
        assert np.all(info.status == oracle.CONVERGED) and np.all(info.relres_true <= 1.1e-8)
    _check_bitwise(bs, systems, rhs, X, infos, 1e-8, 3000)


def test_batched_edges_bitwise(lib):
    """Edge columns and systems: a zero right-hand side (solution 0), a column
    whose initial guess is already the solution (0 passes), a 1 x 1 system, a
    scaled identity (s = 0 after one pass: converged), and maxit = 0."""
    A1 = conv_diff(9, 2, (0.6, -0.3))
    b1, xs1 = manufactured_rhs(A1, 3, seed=3)
    b1[:, 1] = 0.0
    x01 = np.zeros_like(b1)
    x01[:, 0] = 0.25
    x01[:, 2] = xs1[:, 2]
    A2 = CSR(1, np.array([0, 1], np.int32), np.array([0], np.int32), np.array([4.0]))
    b2 = np.array([[2.0, -1.0]])
    n3 = 50
    A3 = CSR(n3, np.arange(n3 + 1, dtype=np.int32), np.arange(n3, dtype=np.int32), np.full(n3, 2.0))
    b3 = np.random.default_rng(4).uniform(-1, 1, (n3, 2))
    systems = [(A1, 3), (A2, 2), (A3, 2)]
    rhs = [b1, b2, b3]
    x0s = [x01, np.zeros_like(b2), np.zeros_like(b3)]
    say("batched edges")
    bs, X, infos = _gpu_solve(lib, systems, rhs, tol=1e-10, maxit=500, x0s=x0s)
    _check_bitwise(bs, systems, rhs, X, infos, 1e-10, 500, x0s=x0s)
    assert np.all(X[0][:, 1] == 0) and list(infos[0].iters[1:]) == [0, 0]
    assert list(infos[1].iters) == [1, 1] and list(infos[2].iters) == [1, 1]
    assert np.all(infos[1].status == oracle.CONVERGED) and np.all(infos[2].status == oracle.CONVERGED)
    # maxit = 0: running columns stop with MAXIT after 0 passes, x unchanged
    bs0, X0, inf0 = _gpu_solve(lib, systems, rhs, tol=1e-10, maxit=0, x0s=x0s)
    assert list(inf0[0].status) == [oracle.MAXIT, oracle.CONVERGED, oracle.CONVERGED]
    assert np.array_equal(X0[0][:, [0, 2]], x01[:, [0, 2]])
    _check_bitwise(bs0, systems, rhs, X0, inf0, 1e-10, 0, x0s=x0s)


def test_batched_empty_rows_and_empty_matrix(lib):
    """Rows without entries and a matrix without any (no column index or
    value array at all: the kernel reads a zero dummy entry): a scaled
    identity with two empty rows whose right-hand side is zero there
    converges in one pass; the zero matrix gives the zero solution for a zero
    right-hand side and BREAKDOWN after one pass (delta = 0) for another one;
    all bit for bit the oracle in the kernel's order."""
    n4 = 40
    keep = np.array([i not in (5, 17) for i in range(n4)])
    rp4 = np.concatenate([[0], np.cumsum(keep)]).astype(np.int32)
    cols4 = np.nonzero(keep)[0].astype(np.int32)
    A4 = CSR(n4, rp4, cols4, np.full(cols4.size, 3.0))
    b4 = np.random.default_rng(6).uniform(-1, 1, (n4, 2))
    b4[~keep] = 0.0
    n5 = 64
    A5 = CSR(n5, np.zeros(n5 + 1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    b5 = np.zeros((n5, 2))
    b5[:, 1] = np.random.default_rng(7).uniform(-1, 1, n5)
    systems = [(A4, 2), (A5, 2)]
    rhs = [b4, b5]
    say("batched empty rows / empty matrix")
    bs, X, infos = _gpu_solve(lib, systems, rhs, tol=1e-10, maxit=50)
    _check_bitwise(bs, systems, rhs, X, infos, 1e-10, 50)
    assert np.all(infos[0].status == oracle.CONVERGED) and list(infos[0].iters) == [1, 1]
    assert list(infos[1].status) == [oracle.CONVERGED, oracle.BREAKDOWN] and list(infos[1].iters) == [0, 1]
    assert np.all(X[1][:, 0] == 0)
    bs.close()


def test_batched_tuner_config_and_determinism(lib):
    """The tuner returns a valid configuration whose solves are bitwise
    reproducible and bitwise the oracle's in that configuration's summation
    order; a hand-set configuration (one workgroup per system) too; invalid
    configurations are rejected."""
    import torch

    systems, rhs = _batch(24, seed=5, nmin=500, nmax=30000)
    say(f"batched tuner: {[(A.n, k) for A, k in systems]}")
    bs = lib.BatchedSolver(systems)
    btens = [torch.from_numpy(b).cuda() for b in rhs]
    best, xt = bs.tune(btens, tol=1e-8, maxit=3000)
    cfg = bs.config()
    say(f"  best {best:.3f} ms, variant {cfg.variant} {lib.batched.variant_info(cfg.variant)}, "
        f"workgroups {cfg.workgroups.tolist()}")
    assert cfg.block == lib.batched.variant_info(cfg.variant)[0] and np.all(cfg.workgroups >= 1) and best > 0
    x1, i1 = bs.solve(btens, tol=1e-8, maxit=3000)
    x2, i2 = bs.solve(btens, tol=1e-8, maxit=3000)
    for s in range(len(systems)):
        assert torch.equal(x1[s], x2[s]) and torch.equal(x1[s], xt[s]), s
        assert np.array_equal(i1[s].iters, i2[s].iters)
    X = [x.cpu().numpy() for x in x1]
    small = sorted(range(len(systems)), key=lambda s: systems[s][0].n)[:6]
    _check_bitwise(bs, systems, rhs, X, i1, 1e-8, 3000, which=small)
    bs.set_config(0, [1] * len(systems))
    _, Xh, ih = _gpu_solve(lib, systems, rhs, tol=1e-8, maxit=3000, solver=bs)
    _check_bitwise(bs, systems, rhs, Xh, ih, 1e-8, 3000, which=small)
    with pytest.raises(lib.BicgstabError):
        bs.set_config(99, [1] * len(systems))
    with pytest.raises(lib.BicgstabError):
        bs.set_config(1, [100000] + [1] * (len(systems) - 1))
    bs.close()


def test_batched_single_workgroup_systems(lib):
    """Every system on one workgroup (its passes synchronised by the
    workgroup barrier alone, no device-wide counter), up to 20,000 rows, to
    tol 1e-8: bit for bit the oracle in that configuration's summation order,
    for a 1024- and a 512-lane variant."""
    systems, rhs = _batch(8, seed=11, nmin=300, nmax=20000)
    say(f"batched single workgroup: {[(A.n, k) for A, k in systems]}")
    bs = lib.BatchedSolver(systems)
    for v in (1, 3):
        bs.set_config(v, [1] * len(systems))
        _, X, infos = _gpu_solve(lib, systems, rhs, tol=1e-8, maxit=3000, solver=bs)
        for info in infos:
            assert np.all(info.status == oracle.CONVERGED)
        _check_bitwise(bs, systems, rhs, X, infos, 1e-8, 3000)
    bs.close()


def test_batched_variants_agree_bitwise(lib):
    """The kernel variants of one block size sum in the same order: with the
    same shares they return identical results, and each matches the oracle in
    that order."""
    from paper_1907_12874_amd.batched import variant_info

    systems, rhs = _batch(10, seed=7)
    bs = lib.BatchedSolver(systems)
    shares = [max(1, min(A.n // 64, 3 + s)) for s, (A, _) in enumerate(systems)]
    by_block = {}
    v = 0
    while True:
        try:
            block, rows, entries, prows = variant_info(v)
        except lib.BicgstabError:
            break
        say(f"variant {v}: block {block}, rows {rows}, entries {entries}, product rows {prows}")
        bs.set_config(v, shares)
        _, X, infos = _gpu_solve(lib, systems, rhs, tol=1e-9, maxit=2000, solver=bs)
        if block in by_block:
            X0, i0 = by_block[block]
            for s in range(len(systems)):
                assert np.array_equal(X[s], X0[s]) and np.array_equal(infos[s].iters, i0[s].iters), (v, s)
        else:
            by_block[block] = (X, infos)
            _check_bitwise(bs, systems, rhs, X, infos, 1e-9, 2000)
        v += 1
    assert v >= 2 and len(by_block) >= 2
    bs.close()


def _row_scaled(systems, seed):
    """The systems with each row scaled by a factor in [0.3, 3]: a diagonal
    that varies from row to row, so Jacobi is not a plain rescaling."""
    rng = np.random.default_rng(seed)
    out = []
    for A, k in systems:
        f = rng.uniform(0.3, 3.0, A.n)
        out.append((CSR(A.n, A.row_ptr, A.col_idx, A.values * np.repeat(f, np.diff(A.row_ptr))), k))
    return out


def test_batched_jacobi_bitwise(lib):
    """Jacobi on every system (12 row-scaled systems, n in [200, 5000], k in
    1..8): 12 fixed passes, then a solve to 1e-8 with initial guesses, bit for
    bit the oracle's Alg. 5 with A M^{-1} folded into the products, summed in
    the kernel's order; every column converges with a true residual <= 1.1
    tol."""
    systems, _ = _batch(12, seed=5)
    systems = _row_scaled(systems, 6)
    rhs = [manufactured_rhs(A, k, 600 + s)[0] for s, (A, k) in enumerate(systems)]
    x0s = [np.random.default_rng(700 + s).uniform(-0.5, 0.5, (A.n, k)) for s, (A, k) in enumerate(systems)]
    say(f"batched jacobi: {[(A.n, k) for A, k in systems]}")
    bs = lib.BatchedSolver(systems, precond="jacobi")
    _, X, infos = _gpu_solve(lib, systems, rhs, tol=0.0, maxit=12, solver=bs)
    _check_bitwise(bs, systems, rhs, X, infos, 0.0, 12, precond="jacobi")
    _, X, infos = _gpu_solve(lib, systems, rhs, tol=1e-8, maxit=3000, x0s=x0s, solver=bs)
    say(f"  passes {[int(i.iters.max()) for i in infos]}")
    for info in infos:
        assert np.all(info.status == oracle.CONVERGED) and np.all(info.relres_true <= 1.1e-8)
    _check_bitwise(bs, systems, rhs, X, infos, 1e-8, 3000, x0s=x0s, precond="jacobi")
    bs.close()


def test_batched_jacobi_rejects(lib):
    """Jacobi with a zero diagonal entry in any system fails at create; a
    method other than the classical one is unsupported."""
    from paper_1907_12874_amd import _lib

    A = conv_diff(6, 2, (1.0, 0.5))
    vals = A.values.copy()
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    vals[(rows == 4) & (A.col_idx == 4)] = 0.0
    with pytest.raises(lib.BicgstabError, match="zero diagonal"):
        lib.BatchedSolver([(A, 1), (CSR(A.n, A.row_ptr, A.col_idx, vals), 2)], precond="jacobi")
    lib.BatchedSolver([(CSR(A.n, A.row_ptr, A.col_idx, vals), 2)]).close()  # fine without a preconditioner
    import ctypes as C

    desc = (_lib.CSRDesc * 1)(_lib.CSRDesc(4, 0, None, None, None))
    ks = (C.c_int32 * 1)(1)
    h = C.c_void_p()
    L = _lib.lib()
    assert L.bicgstab_batched_create(desc, ks, 1, 2, 0, None, C.byref(h)) == _lib.EUNSUPPORTED
    assert L.bicgstab_batched_create(desc, ks, 1, 0, 7, None, C.byref(h)) == _lib.EINVAL


def test_batched_rejects_bad_input(lib):
    import torch

    A = conv_diff(5, 2, (1.0, 0.5))
    bad = CSR(A.n, A.row_ptr.copy(), A.col_idx.copy(), A.values.copy())
    bad.col_idx[3] = A.n + 7
    with pytest.raises(lib.BicgstabError):
        lib.BatchedSolver([(A, 1), (bad, 1)])
    bs = lib.BatchedSolver([(A, 2)])
    with pytest.raises(ValueError):
        bs.solve([torch.zeros(A.n, 3, dtype=torch.float64).cuda()])
    with pytest.raises(ValueError):
        bs.solve([torch.zeros(A.n, 2, dtype=torch.float64).cuda()] * 2)


def test_batched_full_size_64_systems(lib):
    """The batched workload at full size: 64 systems, n log-uniform in
    [1e3, 2e5], k in 1..8, tol 1e-8, tuned. Every column converges with a
    true residual <= 1.1 tol (recomputed on the host); the six smallest
    systems are checked bit for bit against the oracle; four more solves in
    the same configuration repeat the first bit for bit (a stale read of
    another workgroup's rows or partials through a barrier, which once showed
    in about one full-size solve in three, changes the iterates)."""
    import torch

    cfg = config_problem(3, seed=0)
    systems, rhs = cfg["systems"], [b for b, _ in cfg["rhs"]]
    say(f"batched full size: {len(systems)} systems, n {min(A.n for A, _ in systems)}..{max(A.n for A, _ in systems)}")
    bs = lib.BatchedSolver(systems)
    btens = [torch.from_numpy(b).cuda() for b in rhs]
    best, _ = bs.tune(btens, tol=1e-8, maxit=5000)
    xs, infos = bs.solve(btens, tol=1e-8, maxit=5000)
    say(f"  tuned kernel {best:.2f} ms, passes max {max(int(i.iters.max()) for i in infos)}")
    X = [x.cpu().numpy() for x in xs]
    for s, ((A, k), b) in enumerate(zip(systems, rhs)):
        assert np.all(infos[s].status == oracle.CONVERGED), (s, infos[s].status)
        rt = np.linalg.norm(b - A.to_scipy() @ X[s], axis=0) / np.linalg.norm(b, axis=0)
        assert np.all(rt <= 1.1e-8), (s, rt)
        assert np.allclose(infos[s].relres_true, rt, rtol=1e-6), s
    small = sorted(range(len(systems)), key=lambda s: systems[s][0].n)[:6]
    _check_bitwise(bs, systems, rhs, X, infos, 1e-8, 5000, which=small)
    for rep in range(4):
        xr, ir = bs.solve(btens, tol=1e-8, maxit=5000)
        for s in range(len(systems)):
            assert torch.equal(xr[s], xs[s]) and np.array_equal(ir[s].iters, infos[s].iters), (rep, s)
    bs.close()
