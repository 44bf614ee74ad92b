"""The C ABI used from C++ with no Python (tests/c_client/c_abi_client.cpp):
the client builds a 2D convection-diffusion problem, solves it through
bicgstab_create / workspace / solve on the GPU and writes the problem and
the solution to a file. On the GPU its solution must equal, bit for bit, the
Python binding's solve of the same problem (the same library calls), and the
client checks the invalid-argument path itself."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BIN = os.path.join(ROOT, "tests", "c_client", "_bin", "c_abi_client")


def read_problem(path):
    raw = open(path, "rb").read()
    n, k, nnz = np.frombuffer(raw, np.int32, 3)
    off = 12
    rp = np.frombuffer(raw, np.int32, n + 1, off)
    off += 4 * (n + 1)
    col = np.frombuffer(raw, np.int32, nnz, off)
    off += 4 * nnz
    val = np.frombuffer(raw, np.float64, nnz, off)
    off += 8 * nnz
    b = np.frombuffer(raw, np.float64, n * k, off).reshape(n, k)
    off += 8 * n * k
    x = np.frombuffer(raw, np.float64, n * k, off).reshape(n, k)
    assert off + 8 * n * k == len(raw)
    return int(n), int(k), rp, col, val, b, x


def test_client_is_built_and_linked():
    """build() produced the client and its run path finds the in-tree library."""
    if not os.path.exists(BIN):
        pytest.skip("client not built (run __graft_entry__.build())")
    out = subprocess.run(["ldd", BIN], capture_output=True, text=True).stdout
    line = [l for l in out.splitlines() if "libbicgstab.so" in l]
    assert line and "not found" not in line[0] and "paper_1907_12874_amd" in line[0], out


@pytest.mark.gpu
@pytest.mark.parametrize("variant,formulation,precond", [(0, 0, 1), (2, 1, 0), (3, 0, 0), (0, 2, 1)])
def test_client_solve_equals_python_binding(tmp_path, variant, formulation, precond):
    import torch

    import paper_1907_12874_amd as pk
    from paper_1907_12874_amd import _lib

    if not os.path.exists(BIN):
        pytest.skip("client not built (run __graft_entry__.build())")
    out = tmp_path / "problem.bin"
    names = {v: s for s, v in _lib.VARIANTS.items()}, {v: s for s, v in _lib.FORMULATIONS.items()}, \
        {v: s for s, v in _lib.PRECONDS.items()}
    print(f"c client {names[0][variant]}/{names[1][formulation]}/{names[2][precond]}", flush=True)
    r = subprocess.run([BIN, "24", "3", str(variant), str(formulation), str(precond), str(out)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.stdout, r.stderr)
    assert "status=0,0,0" in r.stdout, r.stdout
    n, k, rp, col, val, b, x = read_problem(out)
    assert n == 24 * 24 and k == 3
    s = pk.Solver(torch.from_numpy(rp.copy()), torch.from_numpy(col.copy()), torch.from_numpy(val.copy()), k,
                  variant=names[0][variant], formulation=names[1][formulation], precond=names[2][precond],
                  device="cuda")
    xp, info = s.solve(torch.from_numpy(b.copy()).cuda(), tol=1e-10, maxit=2000)
    assert np.all(info.status == 0)
    assert np.array_equal(xp.cpu().numpy(), x)
    iters = [int(v) for v in r.stdout.split("iters=")[1].split()[0].split(",")]
    assert iters == [int(v) for v in info.iters]
