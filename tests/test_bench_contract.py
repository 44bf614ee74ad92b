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
