"""Builds tests/c_client/_bin/c_abi_client: a C++ program that uses only the
C ABI (include/bicgstab.h) and the HIP runtime, linked against the in-tree
libbicgstab.so (run path relative to the binary)."""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
BIN = os.path.join(HERE, "_bin", "c_abi_client")


def build() -> str:
    cxx = shutil.which("g++") or "/usr/bin/g++"
    os.makedirs(os.path.dirname(BIN), exist_ok=True)
    cmd = [cxx, "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), os.path.join(HERE, "c_abi_client.cpp"),
           "-L", os.path.join(ROOT, "paper_1907_12874_amd"), "-lbicgstab", "-L", "/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../../paper_1907_12874_amd", "-Wl,-rpath,/opt/rocm/lib", "-o", BIN + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building the C ABI client failed:\n{r.stdout}\n{r.stderr}")
    os.replace(BIN + ".tmp", BIN)
    return BIN


if __name__ == "__main__":
    print(build())
