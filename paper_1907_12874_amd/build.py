"""Build libbicgstab.so (gfx950) in-tree with hipcc, and the host executor
libbicgstab_host.so (the same launch plans on the host's cores) with g++ and
OpenMP.

Usage: python -m paper_1907_12874_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libbicgstab.so")
LIB_HOST = os.path.join(PKG, "libbicgstab_host.so")
SOURCES = ["kernels.hip", "spmm.hip", "batched.hip", "api.hip", "plans.cpp"]
HOST_SOURCES = ["host.cpp", "plans.cpp"]
# The host executor: plain C++ (no HIP), no contraction so its updates round
# like the GPU's and the oracle's.
HOST_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-ffp-contract=off", "-I", INCLUDE]

# -ffp-contract=off: no fused multiply-add contraction, so the vector updates
# and products round like their plain definitions. The packed-FP32 feature is
# switched off for all device code (hipcc's host pass warns that it does not
# know the feature; that is harmless).
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-ffp-contract=off",
    "-Xclang",
    "-target-feature",
    "-Xclang",
    "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I",
    INCLUDE,
]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    cc = hipcc()
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def compile_one(src):
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [cc, *FLAGS, "-c", *lang, os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(4, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    build_host(verbose)
    return LIB


def build_host(verbose: bool = False) -> str:
    cxx = shutil.which("g++") or "/usr/bin/g++"
    srcs = [os.path.join(CSRC, s) for s in HOST_SOURCES]
    tmp = LIB_HOST + ".tmp"
    cmd = [cxx, *HOST_FLAGS, "-shared", *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building the host executor failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_HOST)
    return LIB_HOST


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
