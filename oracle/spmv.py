"""Float64 CSR SpMV of the oracle: the C routine ``spmv_ref_f64`` (sequential
row sums in stored order, no fused multiply-add) and a row-by-row Python
evaluation for sampled rows.  Test infrastructure (see the package docstring).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspmv_ref.so")
_lib = None


def build() -> str:
    """Compile spmv_ref.c with gcc (-O2 -ffp-contract=off -fopenmp)."""
    src = os.path.join(_HERE, "spmv_ref.c")
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC",
                           "-shared", "-o", tmp, src])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        lib.spmv_ref_f64.restype = None
        lib.spmv_ref_f64.argtypes = [ctypes.c_int64] + [ctypes.c_void_p] * 5 + [ctypes.c_int]
        lib.spmv_ref_threads.restype = ctypes.c_int
        lib.spmv_ref_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def threads_used(threads: int = 0) -> int:
    return _load().spmv_ref_threads(int(threads))


def spmv(csr, v, threads: int = 0, out=None) -> np.ndarray:
    """w = A v in float64 (all entries, duplicates included, stored order)."""
    lib = _load()
    rp = np.ascontiguousarray(csr.rowptr, dtype=np.int64)
    col = np.ascontiguousarray(csr.col, dtype=np.int32)
    val = np.ascontiguousarray(csr.val, dtype=np.float64)
    x = np.ascontiguousarray(v, dtype=np.float64)
    w = np.empty(csr.n, dtype=np.float64) if out is None else out
    lib.spmv_ref_f64(csr.n, rp.ctypes.data, col.ctypes.data, val.ctypes.data,
                     x.ctypes.data, w.ctypes.data, int(threads))
    return w


def spmv_rows(csr, v, rows) -> np.ndarray:
    """The same sums for selected rows only, in Python float64 arithmetic."""
    out = np.empty(len(rows))
    for o, i in enumerate(rows):
        s = 0.0
        for k in range(int(csr.rowptr[i]), int(csr.rowptr[i + 1])):
            s = s + float(csr.val[k]) * float(v[int(csr.col[k])])
        out[o] = s
    return out
