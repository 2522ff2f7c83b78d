"""Build libnapspmv.so in place with hipcc for gfx950.

``python -m paper_1612_08060_amd.build`` or ``build()``.  The host plan
builder (C++17, OpenMP) and the HIP sources are compiled by one hipcc call
each, in parallel, into a temporary folder, then linked.  Packed-FP32
instructions are disabled for device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

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


FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-fopenmp",
         "-fvisibility=hidden", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def compile_command(src: str, obj: str) -> list:
    return [_hipcc(), *FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]


def link_command(objs: list, out: str) -> list:
    omp = _omp_libdir()
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fopenmp", *objs]
    if omp:
        cmd += [f"-L{omp}", f"-Wl,-rpath,{omp}"]
    return cmd + ["-o", out]


def _run(cmd: list, verbose: bool):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build(verbose: bool = False) -> str:
    tmp = LIB_PATH + ".tmp"
    with tempfile.TemporaryDirectory(prefix="napspmv_build_") as d:
        objs = [os.path.join(d, s + ".o") for s in SOURCES]
        with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
            list(ex.map(lambda so: _run(compile_command(*so), verbose), zip(SOURCES, objs)))
        _run(link_command(objs, tmp), verbose)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
