"""Float64 CSR SpMV of the oracle.  Test infrastructure (see the package
docstring).

spmv        the definition w = A v: each row summed sequentially in stored
            order, no fused multiply-add (C routine spmv_ref_f64).
spmv_split  the same product in the order algorithm standard_spmv of section
            2.1 forms it on each process: local_spmv(A_on_process, v), then
            local_spmv(A_off_process, b_recv) accumulated into w (C routine
            spmv_split_ref_f64).
spmv_split3 the order algorithm NAPSpMV of section 4.3 forms it: the
            on_process, on_node and off_node blocks in turn, each in stored
            order, accumulated into w (C routine spmv_split3_ref_f64).
*_rows      the same sums for sampled rows, in Python float64 arithmetic.
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
        lib.spmv_split_ref_f64.restype = None
        lib.spmv_split_ref_f64.argtypes = ([ctypes.c_int64] + [ctypes.c_void_p] * 5
                                           + [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int])
        lib.spmv_split3_ref_f64.restype = None
        lib.spmv_split3_ref_f64.argtypes = ([ctypes.c_int64] + [ctypes.c_void_p] * 5
                                            + [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                               ctypes.c_int])
        lib.spmv_split_owner_ref_f64.restype = None
        lib.spmv_split_owner_ref_f64.argtypes = ([ctypes.c_int64] + [ctypes.c_void_p] * 6
                                                 + [ctypes.c_int64, ctypes.c_int, ctypes.c_int])
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


def block_starts(n: int, n_p: int, row_starts=None) -> np.ndarray:
    """Row block boundaries: the even contiguous partition of section 2 with
    the remainder rows on the last process, unless given explicitly."""
    if row_starts is not None:
        return np.ascontiguousarray(row_starts, dtype=np.int64)
    b = n // n_p
    s = np.arange(n_p + 1, dtype=np.int64) * b
    s[-1] = n
    return s


def owners(n: int, n_p: int, row_starts=None, strided: bool = False) -> np.ndarray:
    """owner[i]: the process holding row i (and v_i)."""
    if strided:
        return (np.arange(n, dtype=np.int64) % n_p).astype(np.int32)
    st = block_starts(n, n_p, row_starts)
    return (np.searchsorted(st, np.arange(n), side="right") - 1).astype(np.int32)


def spmv_split_owner(csr, v, owner, ppn: int = 1, parts: int = 2, threads: int = 0,
                     out=None) -> np.ndarray:
    """The split-order product for any partition given by owner[i]
    (C routine spmv_split_owner_ref_f64): parts=2 is standard_spmv's order,
    parts=3 NAPSpMV's with nodes of ppn processes."""
    if parts not in (2, 3):
        raise ValueError("parts must be 2 or 3")
    lib = _load()
    rp = np.ascontiguousarray(csr.rowptr, dtype=np.int64)
    col = np.ascontiguousarray(csr.col, dtype=np.int32)
    val = np.ascontiguousarray(csr.val, dtype=np.float64)
    x = np.ascontiguousarray(v, dtype=np.float64)
    own = np.ascontiguousarray(owner, dtype=np.int32)
    w = np.empty(csr.n, dtype=np.float64) if out is None else out
    lib.spmv_split_owner_ref_f64(csr.n, rp.ctypes.data, col.ctypes.data, val.ctypes.data,
                                 x.ctypes.data, w.ctypes.data, own.ctypes.data, int(ppn),
                                 int(parts), int(threads))
    return w


def spmv_split(csr, v, n_p: int, row_starts=None, threads: int = 0, out=None,
               strided: bool = False) -> np.ndarray:
    """w = A v summed as standard_spmv does on every process: the
    on-process block first, then the off-process block, each in stored
    order (C routine spmv_split_ref_f64; strided partitions through
    spmv_split_owner)."""
    if strided:
        return spmv_split_owner(csr, v, owners(csr.n, n_p, strided=True), 1, 2, threads, out)
    lib = _load()
    rp = np.ascontiguousarray(csr.rowptr, dtype=np.int64)
    col = np.ascontiguousarray(csr.col, dtype=np.int32)
    val = np.ascontiguousarray(csr.val, dtype=np.float64)
    x = np.ascontiguousarray(v, dtype=np.float64)
    st = block_starts(csr.n, n_p, row_starts)
    w = np.empty(csr.n, dtype=np.float64) if out is None else out
    lib.spmv_split_ref_f64(csr.n, rp.ctypes.data, col.ctypes.data, val.ctypes.data,
                           x.ctypes.data, w.ctypes.data, int(n_p), st.ctypes.data, int(threads))
    return w


def spmv_split3(csr, v, n_p: int, ppn: int, row_starts=None, threads: int = 0,
                out=None, strided: bool = False) -> np.ndarray:
    """w = A v summed as algorithm NAPSpMV does on every process: the
    on_process block, then the on_node block, then the off_node block, each
    in stored order (C routine spmv_split3_ref_f64; strided partitions
    through spmv_split_owner)."""
    if n_p % ppn:
        raise ValueError("ppn must divide n_p")
    if strided:
        return spmv_split_owner(csr, v, owners(csr.n, n_p, strided=True), ppn, 3, threads, out)
    lib = _load()
    rp = np.ascontiguousarray(csr.rowptr, dtype=np.int64)
    col = np.ascontiguousarray(csr.col, dtype=np.int32)
    val = np.ascontiguousarray(csr.val, dtype=np.float64)
    x = np.ascontiguousarray(v, dtype=np.float64)
    st = block_starts(csr.n, n_p, row_starts)
    w = np.empty(csr.n, dtype=np.float64) if out is None else out
    lib.spmv_split3_ref_f64(csr.n, rp.ctypes.data, col.ctypes.data, val.ctypes.data,
                            x.ctypes.data, w.ctypes.data, int(n_p), st.ctypes.data, int(ppn),
                            int(threads))
    return w


def spmv_split3_rows(csr, v, n_p: int, ppn: int, rows, row_starts=None) -> np.ndarray:
    """spmv_split3 for selected rows only, in Python float64 arithmetic."""
    st = block_starts(csr.n, n_p, row_starts)
    out = np.empty(len(rows))
    for o, i in enumerate(rows):
        r = int(np.searchsorted(st, i, side="right") - 1)
        lo, hi = int(st[r]), int(st[r + 1])
        node = r // ppn
        nlo, nhi = int(st[node * ppn]), int(st[(node + 1) * ppn])
        ks = range(int(csr.rowptr[i]), int(csr.rowptr[i + 1]))
        own = [k for k in ks if lo <= int(csr.col[k]) < hi]
        on_node = [k for k in ks if nlo <= int(csr.col[k]) < nhi and k not in own]
        rest = [k for k in ks if k not in own and k not in on_node]
        s = 0.0
        for k in own + on_node + rest:
            s = s + float(csr.val[k]) * float(v[int(csr.col[k])])
        out[o] = s
    return out


def spmv_split_rows(csr, v, n_p: int, rows, row_starts=None) -> np.ndarray:
    """spmv_split for selected rows only, in Python float64 arithmetic."""
    st = block_starts(csr.n, n_p, row_starts)
    out = np.empty(len(rows))
    for o, i in enumerate(rows):
        r = int(np.searchsorted(st, i, side="right") - 1)
        lo, hi = int(st[r]), int(st[r + 1])
        ks = range(int(csr.rowptr[i]), int(csr.rowptr[i + 1]))
        on = [k for k in ks if lo <= int(csr.col[k]) < hi]
        off = [k for k in ks if not lo <= int(csr.col[k]) < hi]
        s = 0.0
        for k in on + off:
            s = s + float(csr.val[k]) * float(v[int(csr.col[k])])
        out[o] = s
    return out


def spmv_rows(csr, v, rows) -> np.ndarray:
    """The same sums for selected rows only, in Python float64 arithmetic."""
    out = np.empty(len(rows))
    for o, i in enumerate(rows):
        s = 0.0
        for k in range(int(csr.rowptr[i]), int(csr.rowptr[i + 1])):
            s = s + float(csr.val[k]) * float(v[int(csr.col[k])])
        out[o] = s
    return out
