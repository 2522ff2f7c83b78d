"""Build libnapspmv.so in place with hipcc for gfx950.

``python -m paper_1612_08060_amd.build`` or ``build()``.  The host plan
builder (C++17, OpenMP) and the HIP kernels are compiled in one hipcc call.
Packed-FP32 instructions are disabled for device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_PATH = os.path.join(PKG, "libnapspmv.so")
SOURCES = ["plan_build.cpp", "schedule.cpp", "napspmv.hip", "server.hip"]
ARCH = "gfx950"


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found; install ROCm or put hipcc on PATH")


def _omp_libdir() -> str:
    for d in ("/opt/rocm/llvm/lib", "/opt/rocm/lib/llvm/lib"):
        if os.path.exists(os.path.join(d, "libomp.so")):
            return d
    return ""


def command(out: str = LIB_PATH) -> list:
    omp = _omp_libdir()
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-fopenmp", "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", INCLUDE, "-I", CSRC]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    if omp:
        cmd += [f"-L{omp}", f"-Wl,-rpath,{omp}"]
    cmd += ["-o", out]
    return cmd


def build(verbose: bool = False) -> str:
    tmp = LIB_PATH + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
