"""The benchmark's output contract: one JSON line with the headline metric, a
roofline object for the dominant kernel and the oracle's CPU baseline; more
than one GPU is refused before any GPU work."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_kernel_names_follow_the_op_table():
    """The bench names a vector pass by its op id: its list follows the op
    enumeration and the library's op table entry for entry."""
    import re

    sys.path.insert(0, ROOT)
    import bench

    csrc = os.path.join(ROOT, "paper_1907_12874_amd", "csrc")
    plan = open(os.path.join(csrc, "plan.hpp")).read()
    i = plan.index("enum OpId")
    ops = re.findall(r"^\s*(OP_[A-Z0-9_]+)", plan[i:plan.index("OP_NUM", i)], re.M)
    table = open(os.path.join(csrc, "plans.cpp")).read()
    a = table.index("const OpInfo kOps")
    body = table[a:table.index("};", a)]
    assert re.findall(r"// (OP_[A-Z0-9_]+)", body) == ops
    assert re.findall(r'"([a-z0-9_]+)"', body) == bench.OP_NAMES


@pytest.mark.gpu
def test_bench_json_contract():
    """A small run (32^3 grid, k = 4, no sweep or extra sections) prints one
    JSON line carrying every key of the contract."""
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--grid", "32", "--k", "4", "--steps", "2", "--warmup", "1",
           "--no-sweep", "--no-tiers", "--no-host", "--no-random", "--no-tab4"]
    print("bench contract:", " ".join(cmd[1:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for key, typ in (("metric", str), ("value", float), ("unit", str), ("n_gpus", int), ("steps", int),
                     ("warmup", int), ("ms_per_step", float), ("higher_is_better", bool), ("scaling", str),
                     ("dtype", str), ("data", str), ("config", dict), ("roofline", dict), ("cpu_baseline", dict)):
        assert isinstance(d[key], typ), key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["unit"] == "RHS-iterations/s" and d["dtype"] == "f64" and d["vs_baseline"] is None
    assert isinstance(d["config"]["workload"], str) and d["config"]["k"] == 4
    assert d["solve"]["all_converged"]
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    assert roof["achieved"] > 0 and abs(roof["frac"] - roof["achieved"] / roof["peak"]) < 1e-3
    # counter-derived traffic is recorded for the 128^3, k = 32 workload only
    assert roof["traffic"] is None
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["unit"] == "RHS-iterations/s" and cpu["cores"] >= 1
    assert cpu["value"] > 0 and isinstance(cpu["sample"], str)


def _full_size_report():
    """A report shaped like a default full run: every section on, the sweep
    over k = 1..32 for every method and form, Table 4 rows, three random
    sparse widths, the tiers, the 2D system and the host sections."""
    ks = [1, 2, 4, 8, 16, 32]
    sweep = []
    for kk in ks:
        for v in ("classical", "reordered", "pipelined"):
            for f in ("merged", "basic", "fused"):
                sweep.append({"k": kk, "variant": v, "formulation": f, "launches_per_iter": 13,
                              "bytes_per_iter": 14900000000.0, "fixed_rhs_it_per_s": 12345.6,
                              "fixed_GBps": 5370.1, "fixed_ms_per_iter": 2.7812, "model_ms_per_iter": 2.6543,
                              "measured_over_model": 1.012, "solve_ms": 612.33, "solve_iters_max": 216,
                              "solve_rhs_it_per_s": 10400.2, "equal_accuracy": not (v == "reordered" and f == "fused"),
                              "relres_true_max": 9.87654321e-09,
                              "solve_passes_vs_merged": 1.0 if f == "merged" else 1.176})
    gains = {f"{v}_k{kk}": 0.0712 for v in ("classical", "reordered", "pipelined") for kk in ks}
    tab4 = [{"method": m, "m": mm, "basic_ms": 1.2345, "merged_ms": 1.1111, "improvement": 0.1, "model_improvement": 0.12,
             "paper_improvement": 0.1, "basic_GBps": 5000.0, "merged_GBps": 5100.0, "basic_bytes": 1.0e9,
             "merged_bytes": 0.9e9, "paper_basic_ms": 62.0, "paper_merged_ms": 58.0, "merged_speedup_vs_paper": 93.4}
            for m in ("BiCGStab", "IBiCGStab", "PipeBiCGStab", "PBiCGStab", "RBiCGStab", "PPipeBiCGStab")
            for mm in (1, 4, 16)]
    rs = [{"k": kk, "merged": {"ms_per_iter": 4.7512, "rhs_it_per_s": 6730.1, "algorithmic_GBps": 3200.4,
                               "frac_of_peak": 0.4001},
           "basic": {"ms_per_iter": 5.0358, "rhs_it_per_s": 6354.5, "algorithmic_GBps": 3368.2, "frac_of_peak": 0.421},
           "spmm": {"avg_ms": 1.2948, "GBps": 1146.7, "frac_of_peak": 0.1433, "gathered_GBps_no_reuse": 7366.0},
           "solve": {"ms": 65.18, "iters_max": 13, "rhs_it_per_s": 5461.5, "all_converged": True,
                     "relres_true_max": 9.17e-09}, "merging_time_reduction": 0.0502} for kk in (1, 8, 32)]
    small = {"workload": "2D", "passes": 100, "reps": 5,
             "rows": [{"variant": v, "formulation": f, "launches_per_iter": 13, "us_per_iter": 51.23,
                       "us_per_launch": 3.94, "fixed_rhs_it_per_s": 19520.3, "solve_ms": 3.456, "solve_iters": 61,
                       "solve_rhs_it_per_s": 17650.2, "converged": True, "relres_true": 8.1e-11}
                      for v, f in (("classical", "basic"), ("classical", "merged"), ("classical", "fused"),
                                   ("pipelined", "basic"), ("pipelined", "merged"))],
             "persistent_classical_merged": {"solve_ms": 1.234, "kernel_ms": 1.1, "solve_iters": 61,
                                             "us_per_iter": 18.03, "solve_rhs_it_per_s": 49433.1, "converged": True,
                                             "workgroups": 16, "variant": 2}}
    return {
        "metric": "RHS-iterations/s + HBM GB/s, merged vs plain BiCGStab, k=1..32, equal accuracy",
        "value": 10504.2, "unit": "RHS-iterations/s", "n_gpus": 1, "steps": 20, "warmup": 5, "ms_per_step": 610.123,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3D 7-point convection-diffusion 128^3, velocity (1,0.7,0.3), Jacobi, k=32 RHS, "
                               "tol 1e-08, classical merged BiCGStab", "n": 2097152, "nnz": 14581760, "k": 32,
                   "variant": "classical", "formulation": "merged", "precond": "jacobi", "tol": 1e-08},
        "copy_ceiling_GBps": 5312.7,
        "solve": {"iters_min": 190, "iters_max": 216, "relres_true_max": 9.99e-09, "all_converged": True,
                  "bytes_per_iteration": 14900000000.0, "algorithmic_GBps": 5270.3, "frac_of_peak": 0.6588,
                  "stats": {"iterations_enqueued": 224, "launches": 2950, "polls": 28}},
        "roofline": {"bound": "hbm", "achieved": 4151.7, "peak": 8000.0, "unit": "GB/s", "frac": 0.519,
                     "traffic": 1865123456.0, "kernel": "spmm_kernel", "bytes_per_launch": 1257123456.0,
                     "avg_launch_ms": 0.30281234, "source_sha": "0123456789abcdef"},
        "kernels": {f"group_kernel<op{i}>": {"avg_ms": 0.4, "launches_per_iter": 1, "GBps": 5500.0, "share": 0.1}
                    for i in range(12)},
        "seeds": {"1": {"ms": 640.12, "iters_min": 200, "iters_max": 230, "rhs_it_per_s": 10200.1,
                        "all_converged": True, "relres_true_max": 9.9e-09},
                  "2": {"ms": 630.12, "iters_min": 200, "iters_max": 226, "rhs_it_per_s": 10300.1,
                        "all_converged": True, "relres_true_max": 9.9e-09}},
        "sweep": sweep, "merging_time_reduction": gains,
        "fusion_time_reduction_vs_merged": {f"{v}_k{kk}": 0.1012 for v in ("classical", "reordered", "pipelined")
                                            for kk in ks},
        "small_2d": small,
        "gpu_tab4": {"rows": tab4},
        "random_sparse": {"rows": rs},
        "tiers": {"precision": {"fp64": {"ms": 80.03, "err_vs_xstar_max": 2.158362225818514e-09},
                                "fp32_refine": {"ms": 40.49, "err_vs_xstar_max": 1.879629673763007e-09},
                                "speedup_fp32_refine": 1.977,
                                "fp32_refine_tol1e-12": {"ms": 61.23, "err_vs_xstar_max": 2.345678901234e-12}},
                  "batched": {"ms": 387.89, "rhs_it_per_s": 142570.3, "algorithmic_GBps": 2666.6,
                              "speedup_vs_loop": 1.761},
                  "autograd": {"forward_ms": 46.13, "forward_backward_ms": 93.44}},
        "host_tab4": {"rows": tab4},
        "host_executor_baseline": {"value": 608.24, "cores": 16},
        "cpu_baseline": {"value": 33.357, "unit": "RHS-iterations/s", "cores": 1, "kind": "oracle",
                         "sample": "classical/merged/jacobi, column 0 of the same workload, 200 fixed passes (stop test "
                                   "off), 15.0 s; NumPy/SciPy FP64 limited to 1 thread (host has 256 logical CPUs)"},
        "report": "reports/bench_report.json",
    }


def test_compact_line_fits_on_a_full_report():
    """The stdout line composed from a full-size report stays under 4 KB and
    keeps every key of the contract, the roofline and the CPU baseline."""
    sys.path.insert(0, ROOT)
    import bench

    rep = _full_size_report()
    line = bench.compose_line(rep)
    text = json.dumps(line)
    assert len(text) < 4096, len(text)
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
                "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert key in line, key
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in line["roofline"], key
    assert line["config"]["workload"] == rep["config"]["workload"]
    # the section summaries the report has all fit at this size
    for key in ("solve", "seeds", "merged_vs_basic", "fused_vs_merged", "small_2d", "tiers", "random_sparse",
                "report"):
        assert key in line, key
    assert line["sweep_unequal_accuracy"] == [f"reordered/fused/k{kk}" for kk in (1, 2, 4, 8, 16, 32)]
    # and a report with oversized sections still yields a line under the bound
    rep["small_2d"]["rows"] = rep["small_2d"]["rows"] * 40
    for i in range(200):
        rep["random_sparse"]["rows"].append(dict(rep["random_sparse"]["rows"][0], k=100 + i))
    line = bench.compose_line(rep)
    assert len(json.dumps(line)) < 4096
    assert "roofline" in line and "cpu_baseline" in line
