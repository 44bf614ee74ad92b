#!/usr/bin/env python3
"""Benchmark: multi-RHS BiCGStab on one MI355X.

Workload: 3D 7-point convection-diffusion on a 128^3 grid (n = 2,097,152,
14,581,760 nonzeros, FP64 CSR), velocity (1, 0.7, 0.3), Jacobi
preconditioner, k right-hand sides b = A x* with x* ~ U[-1,1], tol 1e-8.

A step is one full solve of all k right-hand sides (start-up passes,
iterations until every column meets the tolerance, exit residual check),
with the matrix, b and x0 already in HBM. The headline is the classical merged
form at k = 32, in RHS-iterations per second (sum over columns of the passes
each column ran, divided by the step time).

Output: the full report (every section below) is written as JSON to
--report (default reports/bench_report.json); stdout gets ONE compact JSON
line (under 4 KB) with the contract's keys and a summary of each section.
Progress lines go to stderr.

The report carries:
  roofline      the dominant kernel of one iteration, timed with HIP events
                around each launch on the stream it runs on, against 8 TB/s;
  cpu_baseline  the CPU oracle, timed on a bounded sample (one column, fixed
                passes) on the host;
  seeds         the headline solve on input seeds 1 and 2 (time, passes);
  sweep         merged vs basic for every method at k = 1..32: fixed-pass
                throughput (RHS-iterations/s, algorithmic GB/s) and solves to
                the same tolerance (equal accuracy, checked per column);
  small_2d      the 64^2 2D system at k = 1 (launch-bound): per-iteration
                time and launches of classical and Pipelined, basic and
                merged, and the same system in the persistent batched kernel;
  gpu_tab4      Table 4 on the GPU with the paper's matrix (200^3 Poisson,
                m = 1, 4, 16): per-iteration times, basic vs merged, of the
                six methods beside the paper's times and gains;
  random_sparse fixed-pass throughput and a solve per k = 1, 8, 32 on a
                random sparse matrix as large as the stencil (15 random
                columns per row), with the sparse product's rate against
                compulsory and gathered bytes;
  tiers         precision (27-point random 100^3, k = 32: FP64 vs FP32 inner
                solves + FP64 refinement at equal final accuracy), batched (64
                systems of log-uniform size in one persistent launch, tuned,
                vs a loop of single solves) and differentiation (64^3
                variable-coefficient diffusion, k = 8: forward solve vs
                forward + adjoint backward through torch.autograd).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBPS = 8000.0
OP_NAMES = [
    "init", "init_p", "zerob", "copy", "fill0", "exit", "dot", "dotself", "sub_alpha", "sub_omega", "xupd", "pupd",
    "c_ppt", "c_xr_rho", "c_r_rho", "r_g3", "r_xzv", "p_g1", "p_g2", "p_g3", "pp_g12", "pp_g34",
    "ref_resid", "ref_scale", "ref_update", "f_sub_alpha_h", "f_pupd_h", "f_xr_rho_h", "ib_init", "ib_g1", "ib_g2",
    "ib_g3", "ib_z", "ib_v", "ib_x", "re_r", "f_xr_rho_d", "f_p_g23", "f_p_g23d", "f_re_xvd", "f_re_xv", "r_dots",
]


def spmm_bytes(n, nnz, k, elem=8):
    """Compulsory bytes of one sparse product: values + column indices, row
    pointers, X read once, Y written once."""
    return (elem + 4) * nnz + 4 * (n + 1) + 2 * elem * n * k


def iteration_bytes(n, nnz, k, traffic, elem=8):
    """Algorithmic bytes of one iteration: two products, the vector passes'
    block reads and writes (Table 2 counting, with the product epilogues'
    operands and scaled copies) and the Jacobi applications (block in, block
    out, diagonal)."""
    blk = elem * n * k
    return (traffic["spmms"] * spmm_bytes(n, nnz, k, elem) + (traffic["reads"] + traffic["writes"]) * blk
            + traffic["precond_apps"] * (2 * blk + elem * n))


def step_bytes(step, n, nnz, k):
    blk = 8 * n * k
    if step["kind"] == "spmm":
        return spmm_bytes(n, nnz, k)
    if step["kind"] == "spmm_dot":
        # the product, plus the epilogue's second operand (dots), its own input
        # row (E_RE4) and / or its Jacobi-scaled copy with the diagonal
        # (E_PREC, E_DOT_W_PREC)
        epi = step["op"]
        extra = (blk if epi in (0, 1, 3, 4) else 0) + (blk if epi == 4 else 0) + (blk + 8 * n if epi in (2, 3) else 0)
        return spmm_bytes(n, nnz, k) + extra
    if step["kind"] == "prec":
        return 2 * blk + 8 * n
    return (step["nin"] + step["nout"]) * blk


def kernel_name(step):
    if step["kind"] == "spmm":
        return "spmm_kernel"
    if step["kind"] == "spmm_dot":
        return "spmm_dot_kernel<" + ("dot_w", "ppt", "prec", "dot_w_prec", "re4")[step["op"]] + ">"
    if step["kind"] == "prec":
        return "prec_kernel"
    return "group_kernel<" + OP_NAMES[step["op"]] + ">"


def roofline_of(solver, b, n, nnz, k, iters=10):
    import torch

    xs = torch.zeros_like(b)
    steps = solver.kernel_times(b, xs, iters=iters)
    agg = {}
    for st in steps:
        name = kernel_name(st)
        a = agg.setdefault(name, {"ms": 0.0, "launches": 0, "bytes": 0.0})
        a["ms"] += st["ms"]
        a["launches"] += 1
        a["bytes"] += step_bytes(st, n, nnz, k)
    total_ms = sum(a["ms"] for a in agg.values())
    total_bytes = sum(a["bytes"] for a in agg.values())
    dom = max(agg, key=lambda nm: agg[nm]["ms"])
    d = agg[dom]
    per_launch_bytes = d["bytes"] / d["launches"]
    per_launch_ms = d["ms"] / d["launches"]
    achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
    kernels = {nm: {"avg_ms": a["ms"] / a["launches"], "launches_per_iter": a["launches"],
                    "GBps": (a["bytes"] / a["launches"]) / (a["ms"] / a["launches"] * 1e-3) / 1e9,
                    "share": a["ms"] / total_ms} for nm, a in agg.items()}
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": None, "kernel": dom,
            "bytes_per_launch": per_launch_bytes, "avg_launch_ms": per_launch_ms}
    it_summary = {"kernel_ms_per_iter": total_ms, "kernel_GBps_per_iter": total_bytes / (total_ms * 1e-3) / 1e9}
    return roof, kernels, it_summary


# Sources that define each kernel family's code and launch shape: counter
# traffic is reported for a kernel only while these are unchanged.
KERNEL_SOURCES = {
    "spmm": ("spmm.hip", "internal.hpp", "reduce.hpp", "plan.hpp", "api.hip"),
    "vector": ("kernels.hip", "method.hpp", "reduce.hpp", "internal.hpp", "plan.hpp", "plans.cpp", "api.hip"),
}


def kernel_family(kernel):
    return "spmm" if kernel.startswith(("spmm", "reduce_runs")) else "vector"


def kernel_source_sha(family="spmm"):
    """Hash of the sources of a kernel family (KERNEL_SOURCES)."""
    import hashlib

    h = hashlib.sha256()
    for fn in KERNEL_SOURCES[family]:
        with open(os.path.join(ROOT, "paper_1907_12874_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_key(grid, k, variant, formulation, precond):
    return f"convdiff{grid}_k{k}_{variant}_{formulation}_{precond}"


def measured_traffic(kernel, key):
    """HBM bytes per launch of `kernel` on workload `key` from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by the same
    counters on a plain 1 GiB copy in the same run), or None if absent or
    taken on other sources of that kernel."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    ent = d.get("workloads", {}).get(key, {}).get("kernels", {}).get(kernel)
    if ent is None or ent.get("source_sha") != kernel_source_sha(kernel_family(kernel)):
        return None
    return ent.get("hbm_bytes_per_launch")


def copy_probe(reps=5):
    """A plain 1 GiB device copy (torch): the known-size kernel that calibrates
    the HBM byte counters, and the practical bandwidth ceiling (read + write
    bytes / time, HIP events on torch's stream, median of `reps`)."""
    import torch

    x = torch.ones(2**27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    del x, y
    ms = sorted(times)[len(times) // 2]
    return round(2 * 2**30 / (ms * 1e-3) / 1e9, 1)


def cpu_baseline(A, b, variant, formulation, precond, budget_s=15.0):
    """The oracle as it stands, one column, fixed passes, single thread."""
    import oracle
    from threadpoolctl import threadpool_limits

    S = A.to_scipy()
    col = np.ascontiguousarray(b[:, 0])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oracle.solve_column(S, col, None, variant, formulation, precond, 0.0, 2)
        t_probe = (time.perf_counter() - t0) / 2
        m = int(max(3, min(200, budget_s / max(t_probe, 1e-6))))
        t0 = time.perf_counter()
        oracle.solve_column(S, col, None, variant, formulation, precond, 0.0, m)
        t = time.perf_counter() - t0
    return {"value": round(m / t, 3), "unit": "RHS-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{variant}/{formulation}/{precond}, column 0 of the same workload, {m} fixed passes "
                      f"(stop test off), {t:.1f} s; NumPy/SciPy FP64 limited to 1 thread "
                      f"(host has {os.cpu_count()} logical CPUs)",
            "seconds": round(t, 2), "passes": m}


def timed(fn, reps=1):
    import torch

    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps, r


def tier_precision(pk, dev, maxit):
    """FP64 vs FP32 + FP64 refinement on the 27-point random matrix, both to a
    true relative residual of 1e-10; errors against the manufactured x*."""
    import torch

    from workloads import config_problem

    cfg = config_problem(2, seed=0)
    A, xs = cfg["A"], cfg["x_star"]
    b = torch.from_numpy(cfg["b"]).to(dev)
    xst = torch.from_numpy(xs).to(dev)
    out = {"workload": f"27-point random 100^3, n={A.n}, nnz={A.nnz}, k={cfg['k']}, tol {cfg['tol']:g}"}
    for prec in ("fp64", "fp32_refine"):
        s = pk.Solver.from_csr(A, cfg["k"], precision=prec, device=dev)
        s.solve(b, tol=cfg["tol"], maxit=maxit)
        t, (x, info) = timed(lambda: s.solve(b, tol=cfg["tol"], maxit=maxit), reps=2)
        err = float(((x - xst).norm(dim=0) / xst.norm(dim=0)).max())
        row = {"ms": round(t * 1e3, 2), "all_converged": bool(np.all(info.status == 0)),
               "relres_true_max": float(info.relres_true.max()), "err_vs_xstar_max": err,
               "rhs_it_per_s": round(float(info.iters.sum()) / t, 1)}
        if prec == "fp32_refine":
            row["outer_corrections_max"] = int(s.refine_outer().max())
            row["inner_passes_max"] = int(info.iters.max())
        else:
            row["passes_max"] = int(info.iters.max())
        out[prec] = row
        s.close()
    out["speedup_fp32_refine"] = round(out["fp64"]["ms"] / out["fp32_refine"]["ms"], 3)
    # refined further: a residual of 1e-12, where the solution error itself
    # falls below 1e-10 (at 1e-10 both precisions stop at the conditioning's
    # ~1e-9 error); the cost of that accuracy
    s = pk.Solver.from_csr(A, cfg["k"], precision="fp32_refine", device=dev)
    s.solve(b, tol=1e-12, maxit=maxit)
    t, (x, info) = timed(lambda: s.solve(b, tol=1e-12, maxit=maxit), reps=2)
    out["fp32_refine_tol1e-12"] = {"ms": round(t * 1e3, 2), "all_converged": bool(np.all(info.status == 0)),
                                   "relres_true_max": float(info.relres_true.max()),
                                   "err_vs_xstar_max": float(((x - xst).norm(dim=0) / xst.norm(dim=0)).max()),
                                   "outer_corrections_max": int(s.refine_outer().max()),
                                   "inner_passes_max": int(info.iters.max())}
    s.close()
    return out


def tier_batched(pk, dev, maxit):
    """64 systems in one persistent launch, tuned, vs a loop of single solves
    (the classical merged single-system path, one system after another)."""
    import torch

    from workloads import config_problem

    cfg = config_problem(3, seed=0)
    systems = cfg["systems"]
    bt = [torch.from_numpy(b).to(dev) for b, _ in cfg["rhs"]]
    bs = pk.BatchedSolver(systems, device=dev)
    t_tune, _ = timed(lambda: bs.tune(bt, tol=cfg["tol"], maxit=maxit))
    t, (xs, infos) = timed(lambda: bs.solve(bt, tol=cfg["tol"], maxit=maxit), reps=2)
    c = bs.config()
    rhs_it = sum(int(i.iters.sum()) for i in infos)
    conv = all(bool(np.all(i.status == 0)) for i in infos)
    byts = 0.0
    for (A, k), i in zip(systems, infos):
        blk = 8.0 * A.n * k
        byts += (2 * (12.0 * A.nnz + 4.0 * A.n + 2 * blk) + 18 * blk) * int(i.iters.max())
    t_loop = 0.0
    for (A, k), b in zip(systems, bt):
        sv = pk.Solver.from_csr(A, k, device=dev)
        sv.solve(b, tol=cfg["tol"], maxit=maxit)
        tl, _ = timed(lambda: sv.solve(b, tol=cfg["tol"], maxit=maxit))
        t_loop += tl
        sv.close()
    bs.close()
    return {"workload": f"{len(systems)} conv-diff systems, n {min(A.n for A, _ in systems)}..{max(A.n for A, _ in systems)},"
                        f" k 1..8 ({sum(k for _, k in systems)} columns), tol {cfg['tol']:g}",
            "ms": round(t * 1e3, 2), "kernel_ms": round(c.last_ms, 2), "rhs_it_per_s": round(rhs_it / t, 1),
            "all_converged": conv, "algorithmic_GBps": round(byts / t / 1e9, 1),
            "variant": c.variant, "workgroups": int(c.workgroups.sum()), "tune_s": round(t_tune, 2),
            "loop_of_single_solves_ms": round(t_loop * 1e3, 2), "speedup_vs_loop": round(t_loop / t, 3)}


def tier_autograd(pk, dev, maxit):
    """Forward solve vs forward + backward (adjoint solve with A^T and the
    pattern gradient) through torch.autograd on the 64^3 diffusion problem."""
    import torch

    from paper_1907_12874_amd import autograd as pag
    from workloads import config_problem
    from workloads import generators as wg

    cfg = config_problem(4, seed=0)
    A = cfg["A"]
    assemble = wg.diffusion_values_torch(A, cfg["g"])
    s = pk.Solver.from_csr(A, cfg["k"], device=dev)
    B = torch.from_numpy(cfg["b"]).to(dev)
    field = torch.tensor(cfg["field"], dtype=torch.float64, device=dev)

    def fwd():
        with torch.no_grad():
            return pag.solve(assemble(field), B, s, tol=cfg["tol"], maxit=maxit)

    def fwd_bwd():
        f = field.clone().requires_grad_(True)
        X = pag.solve(assemble(f), B, s, tol=cfg["tol"], maxit=maxit)
        (X * X).sum().backward()
        return f.grad

    fwd_bwd()
    tf, _ = timed(fwd, reps=2)
    tb, g = timed(fwd_bwd, reps=2)
    s.close()
    return {"workload": f"3D variable-coefficient diffusion 64^3, n={A.n}, k={cfg['k']}, tol {cfg['tol']:g}",
            "forward_ms": round(tf * 1e3, 2), "forward_backward_ms": round(tb * 1e3, 2),
            "backward_over_forward": round((tb - tf) / tf, 3), "grad_finite": bool(torch.isfinite(g).all())}


def random_sparse_section(pk, dev, copy_gbps, ks=(1, 8, 32), passes=20, tol=1e-8, maxit=2000):
    """BiCGStab on a random sparse matrix as large as the stencil (n = 2^21,
    diagonal plus 15 distinct uniformly random columns per row, 1.05x
    dominant diagonal): per k, classical merged and basic with Jacobi at
    fixed passes ((t(2 + passes) - t(2)) / passes: RHS-iterations/s,
    algorithmic GB/s and its fraction of the HBM peak), a merged solve to `tol`, and the sparse product's rate both
    against its compulsory bytes and against the bytes its gathers touch
    when no X row is reused (nnz x 8k: an entry's column is a random row)."""
    import torch

    from workloads import manufactured_rhs, random_sparse

    A = random_sparse(2**21, 15, seed=0)
    n, nnz = A.n, A.nnz
    b_all, _ = manufactured_rhs(A, max(ks), seed=0)
    rows = []
    for kk in ks:
        b = torch.from_numpy(np.ascontiguousarray(b_all[:, :kk])).to(dev)
        x0 = torch.zeros_like(b)
        x = torch.empty_like(b)
        row = {"k": kk}
        for form in ("merged", "basic"):
            sv = pk.Solver.from_csr(A, kk, variant="classical", formulation=form, precond="jacobi", device=dev)
            ib = iteration_bytes(n, nnz, kk, pk.plan_traffic("classical", form, "jacobi"))
            sv.solve(b, x0, tol=0.0, maxit=2, out=x)  # warm-up: prepares the handle
            tp = {}
            for p in (2, 2 + passes):
                torch.cuda.synchronize()
                ta = time.perf_counter()
                sv.solve(b, x0, tol=0.0, maxit=p, out=x)
                torch.cuda.synchronize()
                tp[p] = time.perf_counter() - ta
            tt = (tp[2 + passes] - tp[2]) / passes
            row[form] = {"ms_per_iter": round(tt * 1e3, 4), "rhs_it_per_s": round(kk / tt, 1),
                         "algorithmic_GBps": round(ib / tt / 1e9, 1),
                         "frac_of_peak": round(ib / tt / 1e9 / PEAK_HBM_GBPS, 4)}
            if form == "merged":
                _, kernels, _ = roofline_of(sv, b, n, nnz, kk)
                sp = kernels["spmm_kernel"]
                row["spmm"] = {"avg_ms": round(sp["avg_ms"], 4), "GBps": round(sp["GBps"], 1),
                               "frac_of_peak": round(sp["GBps"] / PEAK_HBM_GBPS, 4),
                               "gathered_GBps_no_reuse": round(
                                   (12.0 * nnz + 4.0 * (n + 1) + 8.0 * nnz * kk + 8.0 * n * kk)
                                   / (sp["avg_ms"] * 1e-3) / 1e9, 1)}
                ta = time.perf_counter()
                _, inf = sv.solve(b, x0, tol=tol, maxit=maxit, out=x)
                torch.cuda.synchronize()
                ts = time.perf_counter() - ta
                row["solve"] = {"ms": round(ts * 1e3, 2), "iters_max": int(inf.iters.max()),
                                "rhs_it_per_s": round(float(inf.iters.sum()) / ts, 1),
                                "all_converged": bool(np.all(inf.status == 0)),
                                "relres_true_max": float(inf.relres_true.max())}
            sv.close()
            del sv
        row["merging_time_reduction"] = round(1 - row["merged"]["ms_per_iter"] / row["basic"]["ms_per_iter"], 4)
        rows.append(row)
        print(f"# random sparse k={kk:2d}: merged {row['merged']['ms_per_iter']:.3f} ms/it "
              f"{row['merged']['algorithmic_GBps']:.0f} GB/s, basic {row['basic']['ms_per_iter']:.3f} ms/it, "
              f"spmm {row['spmm']['avg_ms']:.3f} ms, solve {row['solve']['iters_max']} it",
              file=sys.stderr, flush=True)
    return {"workload": f"random sparse n={n}, nnz={nnz} (diagonal + 15 random columns per row), Jacobi, "
                        f"classical BiCGStab, tol {tol:g}",
            "passes": passes, "copy_ceiling_GBps": copy_gbps, "rows": rows}


TAB4_METHODS = {  # Table 4 rows -> (variant, preconditioner)
    "BiCGStab": ("classical", "none"),
    "IBiCGStab": ("improved", "none"),
    "PipeBiCGStab": ("pipelined", "none"),
    "PBiCGStab": ("classical", "jacobi"),
    "RBiCGStab": ("reordered", "jacobi"),
    "PPipeBiCGStab": ("pipelined", "jacobi"),
}


def host_tab4(pk, grid, reps, threads, run_s=0.25):
    """Table 4 on the host's cores: one iteration of each method, basic and
    merged, for m = 1, 4, 16 right-hand sides of the 7-point Poisson matrix
    (the paper's matrix at grid^3 instead of 200^3), by the host executor of
    the same launch plans. Per-iteration time = the executor's own timing of
    the iteration loop of a fixed-pass solve (set-up and exit excluded) of
    about run_s seconds; basic and merged runs alternate, best of `reps`.
    Reports the time reduction of merging beside the traffic model's
    prediction (1 - bytes merged / bytes basic) and the paper's figures."""
    import json

    # keep OpenMP threads on their cores (read when the executor loads)
    os.environ.setdefault("OMP_PROC_BIND", "close")
    from paper_1907_12874_amd.host import HostSolver
    from workloads import conv_diff

    A = conv_diff(grid, 3, (0.0, 0.0, 0.0))
    n, nnz = A.n, A.nnz
    paper = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")))["table4_merging_effect"]
    rng = np.random.default_rng(0)
    rows = []
    t_all = time.perf_counter()
    for m in (1, 4, 16):
        b = rng.uniform(-1, 1, (n, m))
        for name, (variant, precond) in TAB4_METHODS.items():
            r = {"method": name, "m": m}
            sol, passes, best = {}, {}, {}
            for form in ("basic", "merged"):
                sol[form] = HostSolver.from_csr(A, m, variant=variant, formulation=form, precond=precond,
                                                threads=threads)
                sol[form].solve(b, tol=0.0, maxit=2)
                sec, ran = sol[form].loop_time()
                passes[form] = int(max(2, min(200, run_s / max(sec / max(ran, 1), 1e-6))))
                best[form] = float("inf")
            for _ in range(reps):
                for form in ("basic", "merged"):
                    sol[form].solve(b, tol=0.0, maxit=passes[form])
                    sec, ran = sol[form].loop_time()
                    best[form] = min(best[form], sec / max(ran, 1))
            for form in ("basic", "merged"):
                sol[form].close()
                ib = iteration_bytes(n, nnz, m, pk.plan_traffic(variant, form, precond))
                r[f"{form}_ms"] = round(best[form] * 1e3, 3)
                r[f"{form}_GBps"] = round(ib / best[form] / 1e9, 2)
                r[f"{form}_bytes"] = ib
                r[f"{form}_passes"] = passes[form]
            r["improvement"] = round(1 - r["merged_ms"] / r["basic_ms"], 4)
            r["model_improvement"] = round(1 - r["merged_bytes"] / r["basic_bytes"], 4)
            mi = paper["m"].index(m)
            r["paper_improvement"] = paper["rows"][name][mi][2] / 100.0
            rows.append(r)
            print(f"# host tab4 m={m:2d} {name:14s}: basic {r['basic_ms']:8.2f} ms merged {r['merged_ms']:8.2f} ms "
                  f"imp {r['improvement']:6.1%} (model {r['model_improvement']:5.1%}, paper "
                  f"{r['paper_improvement']:4.0%}), {r['merged_GBps']:.1f} GB/s", file=sys.stderr, flush=True)
    return {"workload": f"7-point Poisson {grid}^3 (n={n}, nnz={nnz}), m = 1, 4, 16, fixed passes; the "
                        f"preconditioned rows use Jacobi (a uniform scaling here: constant diagonal) where the "
                        f"paper used the identity",
            "threads": threads, "reps": reps, "seconds": round(time.perf_counter() - t_all, 1), "rows": rows}


def gpu_tab4(pk, dev, grid=200, passes=10, reps=3):
    """Table 4 on the GPU with the paper's own matrix (7-point Poisson, 200^3)
    and m = 1, 4, 16: per-iteration time of each method, basic and merged,
    as (t(2 + passes) - t(2)) / passes of fixed-pass solves (stop test off;
    start-up passes and exit cancel), each t the best of `reps`, beside the
    paper's per-iteration times on its CPU node and its merging gains."""
    import torch

    from workloads import conv_diff

    A = conv_diff(grid, 3, (0.0, 0.0, 0.0))
    n, nnz = A.n, A.nnz
    with open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")) as f:
        paper = json.load(f)["table4_merging_effect"]
    rng = np.random.default_rng(0)
    rows = []
    t_all = time.perf_counter()
    for m in (1, 4, 16):
        b = torch.from_numpy(rng.uniform(-1, 1, (n, m))).to(dev)
        x0 = torch.zeros_like(b)
        x = torch.empty_like(b)
        for name, (variant, precond) in TAB4_METHODS.items():
            r = {"method": name, "m": m}
            for form in ("basic", "merged"):
                sv = pk.Solver.from_csr(A, m, variant=variant, formulation=form, precond=precond, device=dev)
                # the first solve of a handle also prepares it (graph capture,
                # Alg. 3's transposed matrix): warm up, then the best time of
                # each pass count over `reps`
                sv.solve(b, x0, tol=0.0, maxit=2, out=x)
                tt = {2: float("inf"), 2 + passes: float("inf")}
                for _ in range(reps):
                    for p in tt:
                        torch.cuda.synchronize()
                        ta = time.perf_counter()
                        sv.solve(b, x0, tol=0.0, maxit=p, out=x)
                        torch.cuda.synchronize()
                        tt[p] = min(tt[p], time.perf_counter() - ta)
                best = (tt[2 + passes] - tt[2]) / passes
                sv.close()
                del sv
                ib = iteration_bytes(n, nnz, m, pk.plan_traffic(variant, form, precond))
                r[f"{form}_ms"] = round(best * 1e3, 4)
                r[f"{form}_GBps"] = round(ib / best / 1e9, 1)
                r[f"{form}_bytes"] = ib
            r["improvement"] = round(1 - r["merged_ms"] / r["basic_ms"], 4)
            r["model_improvement"] = round(1 - r["merged_bytes"] / r["basic_bytes"], 4)
            mi = paper["m"].index(m)
            p_basic, p_merged, p_imp = paper["rows"][name][mi]
            r["paper_basic_ms"] = p_basic * 1e3
            r["paper_merged_ms"] = p_merged * 1e3
            r["paper_improvement"] = p_imp / 100.0
            r["merged_speedup_vs_paper"] = round(p_merged / best, 1)
            rows.append(r)
            print(f"# gpu tab4 m={m:2d} {name:14s}: basic {r['basic_ms']:7.3f} ms merged {r['merged_ms']:7.3f} ms "
                  f"imp {r['improvement']:6.1%} (model {r['model_improvement']:5.1%}, paper "
                  f"{r['paper_improvement']:4.0%}), {r['merged_GBps']:.0f} GB/s, "
                  f"{r['merged_speedup_vs_paper']}x the paper's node", file=sys.stderr, flush=True)
        del b, x0, x
    return {"workload": f"7-point Poisson {grid}^3 (n={n}, nnz={nnz}), m = 1, 4, 16, {passes} fixed passes; the "
                        f"preconditioned rows use Jacobi (a uniform scaling here: constant diagonal) where the "
                        f"paper used the identity",
            "paper_source": paper["citation"], "reps": reps,
            "seconds": round(time.perf_counter() - t_all, 1), "rows": rows}


def host_baseline(A, b, variant, formulation, precond, threads, run_s=1.0):
    """The host executor on the headline workload (same matrix, k and
    method): fixed passes on `threads` cores, RHS-iterations/s of the
    iteration loop (best of two runs of about run_s seconds)."""
    from paper_1907_12874_amd.host import HostSolver

    k = b.shape[1]
    hs = HostSolver.from_csr(A, k, variant=variant, formulation=formulation, precond=precond, threads=threads)
    hs.solve(b, tol=0.0, maxit=1)
    sec, ran = hs.loop_time()
    passes = int(max(2, min(100, run_s / max(sec / max(ran, 1), 1e-6))))
    best = float("inf")
    for _ in range(2):
        hs.solve(b, tol=0.0, maxit=passes)
        sec, ran = hs.loop_time()
        best = min(best, sec / max(ran, 1))
    hs.close()
    return {"value": round(k / best, 2), "unit": "RHS-iterations/s", "cores": threads, "kind": "host executor",
            "ms_per_iteration": round(best * 1e3, 3), "passes": passes,
            "sample": f"{variant}/{formulation}/{precond}, all {k} columns of the headline workload, {passes} fixed "
                      f"passes, libbicgstab_host.so on {threads} OpenMP threads"}


def axpby_tab1_gpu(pk, n=10**8, reps=5):
    """Table 1 on the GPU: the three runs of vector updates on n doubles,
    median of `reps` timed with HIP events on torch's stream (the library
    enqueues on it)."""
    import torch

    x = torch.rand(n, dtype=torch.float64, device="cuda")
    y = torch.rand(n, dtype=torch.float64, device="cuda")
    z = torch.rand(n, dtype=torch.float64, device="cuda")
    out = {}
    for run in (1, 2, 3):
        pk.axpby_tab1(run, x, y, z, 0.5, 0.25, 0.125)
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pk.axpby_tab1(run, x, y, z, 0.5, 0.25, 0.125)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        out[f"run{run}_ms"] = round(sorted(ts)[len(ts) // 2], 3)
    moved = {1: 9, 2: 5, 3: 5}
    for run in (1, 2, 3):
        out[f"run{run}_GBps"] = round(moved[run] * n * 8 / (out[f"run{run}_ms"] * 1e-3) / 1e9, 1)
    out["ratio_run1_run2"] = round(out["run1_ms"] / out["run2_ms"], 3)
    out["ratio_run3_run2"] = round(out["run3_ms"] / out["run2_ms"], 3)
    del x, y, z
    return out


def axpby_tab1_host(n=10**8, threads=16, reps=3):
    """Table 1 on the host's cores (the host executor's loops), best of reps."""
    from paper_1907_12874_amd.host import axpby_tab1

    rng = np.random.default_rng(0)
    x, y, z = rng.random(n), rng.random(n), rng.random(n)
    out = {}
    for run in (1, 2, 3):
        axpby_tab1(run, x, y, z, 0.5, 0.25, 0.125, threads=threads)
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            axpby_tab1(run, x, y, z, 0.5, 0.25, 0.125, threads=threads)
            best = min(best, time.perf_counter() - t0)
        out[f"run{run}_ms"] = round(best * 1e3, 2)
    out["ratio_run1_run2"] = round(out["run1_ms"] / out["run2_ms"], 3)
    out["ratio_run3_run2"] = round(out["run3_ms"] / out["run2_ms"], 3)
    out["threads"] = threads
    return out


def small_2d_section(pk, dev, passes=100, reps=5, maxit=3000):
    """The 2D 5-point convection-diffusion system on a 64 x 64 grid (n = 4096,
    k = 1, no preconditioner, tol 1e-10): a launch-bound size, where the merge
    criteria of Section 2.2 show up as kernel launches rather than bytes.
    Per method: fixed-pass time per iteration ((t(2 + passes) - t(2)) /
    passes, best of `reps`), launches per iteration, and a solve to the
    tolerance (best of `reps`). Beside them, the same system through the
    persistent batched kernel (classical merged, one launch for the whole
    solve, autotuned), which has no per-pass launches."""
    import torch

    from workloads import config_problem

    cfg = config_problem(0, seed=0)
    A, tol = cfg["A"], cfg["tol"]
    b = torch.from_numpy(cfg["b"]).to(dev)
    x0 = torch.zeros_like(b)
    x = torch.empty_like(b)
    rows = []
    for variant, form in (("classical", "basic"), ("classical", "merged"), ("classical", "fused"),
                          ("pipelined", "basic"), ("pipelined", "merged"), ("pipelined", "fused")):
        sv = pk.Solver.from_csr(A, 1, variant=variant, formulation=form, precond="none", device=dev)
        tr = pk.plan_traffic(variant, form, "none")
        sv.solve(b, x0, tol=0.0, maxit=2, out=x)
        tt = {2: float("inf"), 2 + passes: float("inf")}
        st = {}
        for _ in range(reps):
            for p in tt:
                torch.cuda.synchronize()
                ta = time.perf_counter()
                sv.solve(b, x0, tol=0.0, maxit=p, out=x)
                torch.cuda.synchronize()
                tt[p] = min(tt[p], time.perf_counter() - ta)
                st[p] = sv.stats()
        per_it = (tt[2 + passes] - tt[2]) / passes
        # kernels per iteration as launched (at this size the alpha / omega
        # steps ride on the next pass, so fewer than the plan's count)
        d_it = st[2 + passes]["iterations_enqueued"] - st[2]["iterations_enqueued"]
        launched = (st[2 + passes]["launches"] - st[2]["launches"]) / max(1, d_it)
        ts = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            ta = time.perf_counter()
            _, inf = sv.solve(b, x0, tol=tol, maxit=maxit, out=x)
            torch.cuda.synchronize()
            ts = min(ts, time.perf_counter() - ta)
        rows.append({"variant": variant, "formulation": form, "launches_per_iter": round(launched, 2),
                     "plan_launches_per_iter": tr["launches"],
                     "us_per_iter": round(per_it * 1e6, 2), "us_per_launch": round(per_it * 1e6 / launched, 2),
                     "fixed_rhs_it_per_s": round(1.0 / per_it, 1), "solve_ms": round(ts * 1e3, 3),
                     "solve_iters": int(inf.iters[0]), "solve_rhs_it_per_s": round(float(inf.iters[0]) / ts, 1),
                     "converged": bool(inf.status[0] == 0), "relres_true": float(inf.relres_true[0])})
        print(f"# small 2d {variant:9s} {form:6s}: {rows[-1]['us_per_iter']:.1f} us/it, {launched:.0f} launches/it, "
              f"solve {rows[-1]['solve_ms']:.2f} ms, {rows[-1]['solve_iters']} it", file=sys.stderr, flush=True)
        sv.close()
    # the persistent batched kernel on this one system
    bs = pk.BatchedSolver([(A, 1)], device=dev)
    bs.tune([b], tol=tol, maxit=maxit)
    tb = float("inf")
    for _ in range(reps):
        t, (_, infos) = timed(lambda: bs.solve([b], tol=tol, maxit=maxit))
        tb = min(tb, t)
    inf = infos[0]
    c = bs.config()
    pers = {"solve_ms": round(tb * 1e3, 3), "kernel_ms": round(c.last_ms, 3), "solve_iters": int(inf.iters[0]),
            "us_per_iter": round(c.last_ms * 1e3 / max(1, int(inf.iters[0])), 2),
            "solve_rhs_it_per_s": round(float(inf.iters[0]) / tb, 1), "converged": bool(inf.status[0] == 0),
            "workgroups": int(c.workgroups.sum()), "variant": c.variant}
    bs.close()
    print(f"# small 2d persistent batched kernel: {pers['solve_ms']:.2f} ms, {pers['solve_iters']} it, "
          f"{pers['us_per_iter']:.1f} us/it on {pers['workgroups']} workgroups", file=sys.stderr, flush=True)
    return {"workload": f"2D 5-point convection-diffusion 64^2, velocity (1,0.5), n={A.n}, nnz={A.nnz}, k=1, "
                        f"no preconditioner, tol {tol:g}",
            "passes": passes, "reps": reps, "rows": rows, "persistent_classical_merged": pers}


def seed_spread(pk, dev, A, k, args, seeds=(1, 2)):
    """The headline solve on the other input seeds (same matrix, x* and so b
    drawn from another seed): time per solve and pass counts."""
    import torch

    from workloads import manufactured_rhs

    out = {}
    s = pk.Solver.from_csr(A, k, variant=args.variant, formulation=args.formulation, precond=args.precond, device=dev)
    for sd in seeds:
        bh, _ = manufactured_rhs(A, k, seed=sd)
        b = torch.from_numpy(bh).to(dev)
        x0 = torch.zeros_like(b)
        x = torch.empty_like(b)
        s.solve(b, x0, tol=args.tol, maxit=args.maxit, out=x)
        t, (_, info) = timed(lambda: s.solve(b, x0, tol=args.tol, maxit=args.maxit, out=x), reps=2)
        out[str(sd)] = {"ms": round(t * 1e3, 2), "iters_min": int(info.iters.min()), "iters_max": int(info.iters.max()),
                        "rhs_it_per_s": round(float(info.iters.sum()) / t, 1),
                        "all_converged": bool(np.all(info.status == 0)),
                        "relres_true_max": float(info.relres_true.max())}
        print(f"# seed {sd}: {out[str(sd)]['ms']:.1f} ms/solve, iters {out[str(sd)]['iters_min']}.."
              f"{out[str(sd)]['iters_max']}, {out[str(sd)]['rhs_it_per_s']:.0f} RHS-it/s", file=sys.stderr, flush=True)
        del b, x0, x
    s.close()
    return out


LINE_MAX_BYTES = 4000


def compose_line(rep):
    """The one JSON line printed last on stdout: the contract's keys, the
    roofline and CPU baseline, and a compact summary of every section of the
    full report (which goes to a file). Kept under LINE_MAX_BYTES: optional
    summaries are dropped, least important first, if it would grow past it."""
    keys = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
            "vs_baseline", "dtype", "data")
    line = {k: rep[k] for k in keys if k in rep}
    cfg = rep.get("config", {})
    line["config"] = {k: cfg[k] for k in ("workload", "n", "nnz", "k", "variant", "formulation", "precond", "tol")
                      if k in cfg}
    if "roofline" in rep:
        r = rep["roofline"]
        line["roofline"] = {k: r[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                                              "bytes_per_launch", "avg_launch_ms") if k in r}
    if "cpu_baseline" in rep:
        c = rep["cpu_baseline"]
        line["cpu_baseline"] = {k: c[k] for k in ("value", "unit", "cores", "kind", "sample") if k in c}
    opt = []  # (key, value), most important first
    if "solve" in rep:
        s = rep["solve"]
        opt.append(("solve", {k: s[k] for k in ("iters_min", "iters_max", "all_converged", "relres_true_max",
                                                "algorithmic_GBps", "frac_of_peak") if k in s}))
    if "copy_ceiling_GBps" in rep:
        opt.append(("copy_GBps", rep["copy_ceiling_GBps"]))
    if "seeds" in rep:
        opt.append(("seeds", {sd: [v["ms"], v["iters_max"], v["all_converged"]] for sd, v in rep["seeds"].items()}))
    if "merging_time_reduction" in rep:
        # per method, the time reduction of merged over basic at each k of the sweep
        ks = sorted({r["k"] for r in rep.get("sweep", [])})
        g = rep["merging_time_reduction"]
        opt.append(("merged_vs_basic", {"k": ks, **{v: [g.get(f"{v}_k{kk}") for kk in ks]
                                                    for v in ("classical", "reordered", "pipelined", "improved")
                                                    if any(f"{v}_k{kk}" in g for kk in ks)}}))
        f = rep.get("fusion_time_reduction_vs_merged", {})
        if f:
            opt.append(("fused_vs_merged", {v: [f.get(f"{v}_k{kk}") for kk in ks]
                                            for v in ("classical", "reordered", "pipelined")
                                            if any(f"{v}_k{kk}" in f for kk in ks)}))
        bad = [f"{r['variant']}/{r['formulation']}/k{r['k']}" for r in rep.get("sweep", []) if not r["equal_accuracy"]]
        opt.append(("sweep_unequal_accuracy", bad))
        gap = {f"{r['variant'][:4]}/{r['formulation']}/k{r['k']}": r["solve_passes_vs_merged"]
               for r in rep.get("sweep", []) if abs(r.get("solve_passes_vs_merged", 1.0) - 1.0) > 0.05}
        opt.append(("sweep_solve_pass_gap", gap))
    if "small_2d" in rep:
        sm = rep["small_2d"]
        opt.append(("small_2d", {**{f"{r['variant'][:4]}_{r['formulation']}": [r["us_per_iter"], r["launches_per_iter"],
                                                                                 r["solve_ms"], r["solve_iters"]]
                                    for r in sm["rows"]},
                                 "persistent": [sm["persistent_classical_merged"]["us_per_iter"],
                                                sm["persistent_classical_merged"]["solve_ms"],
                                                sm["persistent_classical_merged"]["solve_iters"]]}))
    if "tiers" in rep:
        t = rep["tiers"]
        tl = {}
        if "precision" in t:
            p = t["precision"]
            tl["precision"] = {"fp64_ms": p["fp64"]["ms"], "fp32_refine_ms": p["fp32_refine"]["ms"],
                               "speedup": p["speedup_fp32_refine"],
                               "err_vs_xstar": [p["fp64"]["err_vs_xstar_max"], p["fp32_refine"]["err_vs_xstar_max"]]}
            if "fp32_refine_tol1e-12" in p:
                tl["precision"]["tol1e-12"] = [p["fp32_refine_tol1e-12"]["ms"],
                                               p["fp32_refine_tol1e-12"]["err_vs_xstar_max"]]
        if "batched" in t:
            bt = t["batched"]
            tl["batched"] = {"ms": bt["ms"], "rhs_it_per_s": bt["rhs_it_per_s"], "GBps": bt["algorithmic_GBps"],
                             "speedup_vs_loop": bt["speedup_vs_loop"]}
        if "autograd" in t:
            a = t["autograd"]
            tl["autograd"] = {"fwd_ms": a["forward_ms"], "fwd_bwd_ms": a["forward_backward_ms"]}
        opt.append(("tiers", tl))
    if "random_sparse" in rep:
        opt.append(("random_sparse", {f"k{r['k']}": [r["merged"]["ms_per_iter"], r["merged"]["frac_of_peak"],
                                                     r["spmm"]["frac_of_peak"]]
                                      for r in rep["random_sparse"]["rows"]}))
    if "gpu_tab4" in rep:
        opt.append(("gpu_tab4_imp", {f"{r['method']}_m{r['m']}": r["improvement"] for r in rep["gpu_tab4"]["rows"]}))
    if "host_executor_baseline" in rep:
        h = rep["host_executor_baseline"]
        opt.append(("host_executor", {"value": h["value"], "cores": h["cores"]}))
    if "report" in rep:
        opt.append(("report", rep["report"]))
    for k, v in opt:
        line[k] = v
    # drop the least important summaries until the line fits
    for k, _ in reversed(opt):
        if len(json.dumps(line)) <= LINE_MAX_BYTES:
            break
        if k != "report":
            line.pop(k, None)
    return line


def profile_run(pk, dev, what, maxit, k=32):
    """One workload after a warm-up, for kernel traces and counter runs under
    rocprofv3 (after the 1 GiB device copy that calibrates the byte
    counters): the precision tier's matrix solved in FP64 or FP32 + FP64
    refinement, the batched tier's 64 systems (autotuned, then solved), or
    the random sparse matrix (n = 2^21, 15 random columns per row) at k
    right-hand sides, classical merged with Jacobi, `maxit` fixed passes."""
    import torch

    from workloads import config_problem

    copy_probe(reps=1)
    if what == "random":
        from workloads import manufactured_rhs, random_sparse

        A = random_sparse(2**21, 15, seed=0)
        b = torch.from_numpy(np.ascontiguousarray(manufactured_rhs(A, k, seed=0)[0])).to(dev)
        s = pk.Solver.from_csr(A, k, variant="classical", formulation="merged", precond="jacobi", device=dev)
        s.solve(b, tol=0.0, maxit=2)
        t, _ = timed(lambda: s.solve(b, tol=0.0, maxit=maxit))
        print("random sparse k", k, "ms", round(t * 1e3, 2), "passes", maxit, flush=True)
        s.close()
    elif what in ("fp64", "fp32_refine"):
        cfg = config_problem(2, seed=0)
        b = torch.from_numpy(cfg["b"]).to(dev)
        s = pk.Solver.from_csr(cfg["A"], cfg["k"], precision=what, device=dev)
        s.solve(b, tol=cfg["tol"], maxit=maxit)
        t, (_, info) = timed(lambda: s.solve(b, tol=cfg["tol"], maxit=maxit))
        print(what, "ms", round(t * 1e3, 2), "passes", int(info.iters.max()), flush=True)
        s.close()
    else:
        cfg = config_problem(3, seed=0)
        rhs = [torch.from_numpy(b).to(dev) for b, _ in cfg["rhs"]]
        bs = pk.BatchedSolver(cfg["systems"], device=dev)
        bs.tune(rhs, tol=cfg["tol"], maxit=maxit)
        t, _ = timed(lambda: bs.solve(rhs, tol=cfg["tol"], maxit=maxit))
        print("batched ms", round(t * 1e3, 2), "config", bs.config(), flush=True)
        bs.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--variant", default="classical")
    ap.add_argument("--formulation", default="merged")
    ap.add_argument("--precond", default="jacobi")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--no-tiers", action="store_true")
    ap.add_argument("--no-random", action="store_true", help="skip the random sparse matrix section")
    ap.add_argument("--no-tab4", action="store_true", help="skip Table 4 on the GPU (200^3 Poisson)")
    ap.add_argument("--no-small", action="store_true", help="skip the 64^2 2D system (k = 1, launch-bound)")
    ap.add_argument("--no-seeds", action="store_true", help="skip the headline solve on input seeds 1 and 2")
    ap.add_argument("--report", default=os.path.join(ROOT, "reports", "bench_report.json"),
                    help="where the full report goes (JSON); stdout gets one compact line")
    ap.add_argument("--profile-run", choices=("fp64", "fp32_refine", "batched", "random"),
                    help="run one workload after a warm-up and exit without the JSON line (the command behind "
                         "the tier kernel traces and the counter runs; 'random' takes --k and --maxit passes)")
    ap.add_argument("--sweep-passes", type=int, default=20)
    ap.add_argument("--no-host", action="store_true", help="skip the host-CPU Table 4 section")
    ap.add_argument("--host-grid", type=int, default=160)
    ap.add_argument("--host-reps", type=int, default=3)
    ap.add_argument("--sweep-k", default="1,2,4,8,16,32")
    ap.add_argument("--maxit", type=int, default=5000, help="pass cap (lower it for profiled runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="(kept for the profiling commands: the 1 GiB copy that calibrates the counters always runs)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library solves on one device and has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1907_12874_amd as pk
    from workloads import config_problem

    pk.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.profile_run:
        profile_run(pk, dev, args.profile_run, min(args.maxit, 3000), k=args.k)
        return
    copy_gbps = copy_probe()
    print(f"# plain 1 GiB device copy: {copy_gbps} GB/s (read + write)", file=sys.stderr, flush=True)
    t_gen = time.perf_counter()
    cfg = config_problem(1, seed=0, k=args.k, scale=args.grid)
    A = cfg["A"]
    n, nnz, k = A.n, A.nnz, args.k
    print(f"# workload 3D 7-point {args.grid}^3: n={n} nnz={nnz} k={k} (generated in {time.perf_counter() - t_gen:.1f} s)",
          file=sys.stderr, flush=True)
    b = torch.from_numpy(cfg["b"]).to(dev)
    x0 = torch.zeros_like(b)
    x = torch.empty_like(b)

    # ---------------------------------------------------------- headline
    s = pk.Solver.from_csr(A, k, variant=args.variant, formulation=args.formulation, precond=args.precond,
                           device=dev)
    for _ in range(args.warmup):
        s.solve(b, x0, tol=args.tol, maxit=args.maxit, out=x)
    torch.cuda.synchronize()
    iters_total = 0
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, info = s.solve(b, x0, tol=args.tol, maxit=args.maxit, out=x)
        infos.append(info)
        iters_total += int(info.iters.sum())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    info = infos[-1]
    if not np.all(info.status == 0) or not np.all(info.relres_true <= 1.1 * args.tol):
        print(f"# WARNING: not every column converged: status {info.status}", file=sys.stderr)
    traffic = pk.plan_traffic(args.variant, args.formulation, args.precond)
    it_bytes = iteration_bytes(n, nnz, k, traffic)
    value = iters_total / elapsed
    ms_per_step = elapsed / args.steps * 1e3
    max_iters = int(info.iters.max())
    solve_gbps = max_iters * it_bytes / (ms_per_step * 1e-3) / 1e9
    print(f"# headline: {ms_per_step:.1f} ms/solve, iters {int(info.iters.min())}..{max_iters}, "
          f"{value:.0f} RHS-it/s, {solve_gbps:.0f} GB/s algorithmic", file=sys.stderr, flush=True)

    out = {
        "metric": "RHS-iterations/s + HBM GB/s, merged vs plain BiCGStab, k=1..32, equal accuracy",
        "value": round(value, 1),
        "unit": "RHS-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"3D 7-point convection-diffusion {args.grid}^3, velocity (1,0.7,0.3), Jacobi, "
                               f"k={k} RHS, tol {args.tol:g}, {args.variant} {args.formulation} BiCGStab",
                   "n": n, "nnz": nnz, "k": k, "variant": args.variant, "formulation": args.formulation,
                   "precond": args.precond, "tol": args.tol},
        "copy_ceiling_GBps": copy_gbps,
        "solve": {"iters_min": int(info.iters.min()), "iters_max": max_iters,
                  "relres_true_max": float(info.relres_true.max()), "all_converged": bool(np.all(info.status == 0)),
                  "bytes_per_iteration": it_bytes, "algorithmic_GBps": round(solve_gbps, 1),
                  "frac_of_peak": round(solve_gbps / PEAK_HBM_GBPS, 4), "stats": s.stats()},
    }

    if not args.no_roofline:
        roof, kernels, it_summary = roofline_of(s, b, n, nnz, k)
        roof["traffic"] = measured_traffic(roof["kernel"],
                                           traffic_key(args.grid, k, args.variant, args.formulation, args.precond))
        roof["source_sha"] = kernel_source_sha(kernel_family(roof["kernel"]))
        out["roofline"] = roof
        out["kernels"] = kernels
        out["iteration"] = it_summary
        print(f"# roofline: {roof['kernel']} {roof['achieved']:.0f} GB/s ({roof['frac']:.1%})", file=sys.stderr,
              flush=True)

    # ------------------------------------------------------ other seeds
    if not args.no_seeds:
        out["seeds"] = seed_spread(pk, dev, A, k, args)

    # ------------------------------------------------------------- sweep
    if not args.no_sweep:
        sweep = []
        ks = [int(v) for v in args.sweep_k.split(",") if v]
        for kk in ks:
            bk = b[:, :kk].contiguous() if kk <= k else None
            if bk is None:
                continue
            x0k = torch.zeros_like(bk)
            xk = torch.empty_like(bk)
            variants = ("classical", "reordered", "pipelined") + (("improved",) if args.precond == "none" else ())
            for variant in variants:
                for form in ("merged", "basic", "fused") if variant != "improved" else ("merged", "basic"):
                    sv = pk.Solver.from_csr(A, kk, variant=variant, formulation=form, precond=args.precond, device=dev)
                    tr = pk.plan_traffic(variant, form, args.precond)
                    ib = iteration_bytes(n, nnz, kk, tr)
                    # fixed passes (stop test off): per-iteration time as
                    # (t(2 + P) - t(2)) / P, so start-up passes and the exit
                    # check cancel; a warm-up solve prepares the handle first
                    sv.solve(bk, x0k, tol=0.0, maxit=2, out=xk)
                    tp, stp = {}, {}
                    for p in (2, 2 + args.sweep_passes):
                        torch.cuda.synchronize()
                        ta = time.perf_counter()
                        sv.solve(bk, x0k, tol=0.0, maxit=p, out=xk)
                        torch.cuda.synchronize()
                        tp[p] = time.perf_counter() - ta
                        stp[p] = sv.stats()
                    tt = tp[2 + args.sweep_passes] - tp[2]
                    d_it = stp[2 + args.sweep_passes]["iterations_enqueued"] - stp[2]["iterations_enqueued"]
                    launched = (stp[2 + args.sweep_passes]["launches"] - stp[2]["launches"]) / max(1, d_it)
                    # solve to the tolerance: equal accuracy
                    ta = time.perf_counter()
                    _, inf = sv.solve(bk, x0k, tol=args.tol, maxit=min(args.maxit, 2000), out=xk)
                    torch.cuda.synchronize()
                    ts = time.perf_counter() - ta
                    row = {"k": kk, "variant": variant, "formulation": form, "launches_per_iter": round(launched, 2),
                           "plan_launches_per_iter": tr["launches"],
                           "bytes_per_iter": ib,
                           "fixed_rhs_it_per_s": round(kk * args.sweep_passes / tt, 1),
                           "fixed_GBps": round(args.sweep_passes * ib / tt / 1e9, 1),
                           "fixed_ms_per_iter": round(tt / args.sweep_passes * 1e3, 4),
                           # Tab. 5/6's model T = bytes / B with B the measured device copy
                           "model_ms_per_iter": round(ib / (copy_gbps * 1e9) * 1e3, 4),
                           "measured_over_model": round(tt / args.sweep_passes / (ib / (copy_gbps * 1e9)), 3),
                           "solve_ms": round(ts * 1e3, 2), "solve_iters_max": int(inf.iters.max()),
                           "solve_rhs_it_per_s": round(float(inf.iters.sum()) / ts, 1),
                           "equal_accuracy": bool(np.all(inf.status == 0) and np.all(inf.relres_true <= 1.1 * args.tol)),
                           "relres_true_max": float(inf.relres_true.max())}
                    sweep.append(row)
                    print(f"# sweep k={kk:2d} {variant:9s} {form:6s}: {row['fixed_ms_per_iter']:.3f} ms/it "
                          f"{row['fixed_GBps']:.0f} GB/s | solve {row['solve_ms']:.0f} ms, "
                          f"{row['solve_iters_max']} it", file=sys.stderr, flush=True)
                    sv.close()
                    del sv
        # A solve's time also depends on how many passes it took, and forms
        # that differ only in rounding order stop at different pass counts
        # (BiCGStab amplifies summation-order differences near the
        # tolerance): flag each form's solve pass count against the merged
        # form's, so solve times are not read as per-pass speed.
        for r in sweep:
            m = [q for q in sweep if q["k"] == r["k"] and q["variant"] == r["variant"] and q["formulation"] == "merged"]
            if m and m[0]["solve_iters_max"] > 0:
                r["solve_passes_vs_merged"] = round(r["solve_iters_max"] / m[0]["solve_iters_max"], 3)
        out["sweep"] = sweep
        gains, fusion = {}, {}
        for kk in ks:
            for variant in ("classical", "reordered", "pipelined", "improved"):
                m = [r for r in sweep if r["k"] == kk and r["variant"] == variant]
                mb = {r["formulation"]: r for r in m}
                if "merged" in mb and "basic" in mb:
                    gains[f"{variant}_k{kk}"] = round(1 - mb["merged"]["fixed_ms_per_iter"] / mb["basic"]["fixed_ms_per_iter"], 4)
                if "fused" in mb and "merged" in mb:
                    fusion[f"{variant}_k{kk}"] = round(1 - mb["fused"]["fixed_ms_per_iter"] / mb["merged"]["fixed_ms_per_iter"], 4)
        out["merging_time_reduction"] = gains
        out["fusion_time_reduction_vs_merged"] = fusion
        # the paper's own merging gains (Tab. 4, its CPU node) beside ours
        with open(os.path.join(ROOT, "tests", "golden", "paper_tables.json")) as f:
            tab4 = json.load(f)["table4_merging_effect"]
        tab4_names = {"jacobi": {"classical": "PBiCGStab", "reordered": "RBiCGStab", "pipelined": "PPipeBiCGStab"},
                      "none": {"classical": "BiCGStab", "pipelined": "PipeBiCGStab", "improved": "IBiCGStab"}}
        out["merging_time_reduction_paper"] = {
            "source": tab4["citation"], "m": tab4["m"],
            **{v: [r[2] / 100.0 for r in tab4["rows"][nm]] for v, nm in tab4_names.get(args.precond, {}).items()}}

    # ------------------------------------------- the 64^2 2D system, k = 1
    if not args.no_small:
        out["small_2d"] = small_2d_section(pk, dev)

    # ------------------------------------------- Table 4 on the GPU
    if not args.no_tab4:
        out["gpu_tab4"] = gpu_tab4(pk, dev)

    # ------------------------------------------------------ random sparse
    if not args.no_random:
        out["random_sparse"] = random_sparse_section(pk, dev, copy_gbps, tol=args.tol)

    # -------------------------------------------------------------- tiers
    if not args.no_tiers:
        tiers = {}
        for name, fn in (("precision", tier_precision), ("batched", tier_batched), ("autograd", tier_autograd)):
            tiers[name] = fn(pk, dev, args.maxit)
            print(f"# tier {name}: {json.dumps(tiers[name])}", file=sys.stderr, flush=True)
        out["tiers"] = tiers

    # ------------------------------------------------------------ Table 1
    tab1 = {"n": 10**8, "paper_ratio_run1_run2": {"Lomonosov": round(207 / 117, 3),
                                                   "Lomonosov-2": round(125 / 71, 3)},
            "traffic_ratio_run1_run2": 1.8, "gpu": axpby_tab1_gpu(pk)}
    print(f"# table 1 gpu: {json.dumps(tab1['gpu'])}", file=sys.stderr, flush=True)
    if not args.no_host:
        tab1["host"] = axpby_tab1_host(threads=max(1, min(16, os.cpu_count() or 1)))
        print(f"# table 1 host: {json.dumps(tab1['host'])}", file=sys.stderr, flush=True)
    out["axpby_tab1"] = tab1

    # ------------------------------------------- host cores: Table 4
    if not args.no_host:
        threads = max(1, min(16, os.cpu_count() or 1))
        out["host_tab4"] = host_tab4(pk, args.host_grid, args.host_reps, threads)
        out["host_executor_baseline"] = host_baseline(A, cfg["b"], args.variant, args.formulation, args.precond,
                                                      threads)
        print(f"# host executor ({threads} threads): {out['host_executor_baseline']['value']} RHS-it/s",
              file=sys.stderr, flush=True)

    # ------------------------------------------------------- CPU baseline
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(A, cfg["b"], args.variant, args.formulation, args.precond)
        print(f"# cpu baseline: {out['cpu_baseline']['value']} RHS-it/s", file=sys.stderr, flush=True)

    # the full report to a file, one compact line (under 4 KB) to stdout
    try:
        os.makedirs(os.path.dirname(os.path.abspath(args.report)), exist_ok=True)
        with open(args.report, "w") as f:
            json.dump(out, f, indent=1)
        out["report"] = os.path.relpath(os.path.abspath(args.report), ROOT)
    except OSError as e:
        print(f"# could not write the full report: {e}", file=sys.stderr, flush=True)
    print(json.dumps(compose_line(out)), flush=True)


if __name__ == "__main__":
    main()
