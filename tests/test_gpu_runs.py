"""Parity of the vector-run product kernels with the oracle, on an MI355X.

The on-process product loads aligned runs of 2, 4 or 8 entries per lane
(float64, float32, bfloat16 values), the off-process product runs of 16
bytes of values laid out by the host in load order, with each entry's ghost
position and slot packed in one word where the block allows it, and
off-process blocks whose ghost positions span less than 65536 read 16-bit
offsets from a per-block base.  These tests aim at the edges of those
layouts:

* row blocks whose first entry is not aligned, rows of exactly the block
  capacity and a few entries either side of it (single-row blocks whose
  aligned span exceeds the capacity, and longer rows, take the chunked
  path), empty rows and processes without off-process entries, at every
  block size;
* one plan holding both narrow off-process blocks (halos read from the
  neighbouring process only) and wide ones (columns drawn from the whole
  matrix, more than 65536 ghost positions apart);
* one plan holding packed blocks and blocks whose lane groups read ghost
  positions 2^19 or more apart (int32 positions and slots);

float64 w bitwise equal to the oracle's split-order product (both modes),
float32 and bfloat16 values within 1e-5 and 2e-2 normwise of the float64
oracle.
"""
import numpy as np
import pytest
import torch

import paper_1612_08060_amd as nap
from oracle import spmv as oracle_spmv
from workloads import CSR, bf16_bits, to_f32, vec_normal

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = {"f32": 1e-5, "bf16": 2e-2}


def _csr_from_rows(n, rows, seed):
    lens = np.array([len(r) for r in rows], dtype=np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    col = np.concatenate([np.asarray(r, dtype=np.int32) for r in rows]) if rowptr[-1] else \
        np.zeros(0, dtype=np.int32)
    return CSR(n, rowptr, col, vec_normal(int(rowptr[-1]), seed))


def _apply(a, v, n_p, ppn, mode, dtype, params):
    vals = {"f64": a.val, "f32": to_f32(a.val), "bf16": bf16_bits(a.val)}[dtype]
    p = nap.Plan(a.rowptr, a.col, vals, a.n, n_p, ppn, mode=mode, dtype=dtype)
    for k, x in params.items():
        p.set_param(k, x)
    tv = torch.from_numpy(v if dtype == "f64" else to_f32(v)).to(DEV)
    w = torch.full_like(tv, float("nan"))
    p.apply(tv, w)
    torch.cuda.synchronize()
    p.close()
    return w.cpu().numpy().astype(np.float64)


def _relerr(w, ref):
    return np.linalg.norm(w - ref) / max(np.linalg.norm(ref), 1e-300)


def _boundary_matrix(cap, seed):
    """8 processes of 600 rows: short rows of 0..40 entries (about half of
    them off-process), and in processes 1 and 5 single rows of cap - 9 ..
    cap + 3 entries, so that blocks start at every alignment and some
    single-row blocks have an aligned span just over the capacity;
    process 3 has no off-process entry at all."""
    rng = np.random.default_rng(seed)
    n_p, per = 8, 600
    n = n_p * per
    rows = []
    for i in range(n):
        t = i // per
        lo, hi = t * per, (t + 1) * per
        if t in (1, 5) and (i - lo) % 50 == 7:
            m = cap - 9 + ((i - lo) // 50) % 13
        else:
            m = int(rng.integers(0, 41))
        if t == 3:
            cols = rng.integers(lo, hi, size=m)
        else:
            far = rng.random(m) < 0.5
            cols = np.where(far, rng.integers(0, n, size=m), rng.integers(lo, hi, size=m))
        rows.append(cols)
    return _csr_from_rows(n, rows, seed + 1), n_p


@pytest.mark.parametrize("cap", [1024, 2048, 4096, 8192])
def test_run_block_boundaries(cap):
    a, n_p = _boundary_matrix(cap, seed=cap)
    v = vec_normal(a.n, 7)
    split = oracle_spmv.spmv_split(a, v, n_p)
    ref = oracle_spmv.spmv(a, v)
    for rcap in sorted({1024, cap}):
        params = {"block_nnz": cap, "remote_nnz": rcap}
        for mode in ("standard", "nap"):
            w = _apply(a, v, n_p, 2, mode, "f64", params)
            assert np.array_equal(w, split), (cap, rcap, mode)
        for dt in ("f32", "bf16"):
            w = _apply(a, v, n_p, 2, "standard", dt, params)
            assert _relerr(w, ref) <= TOL[dt], (cap, rcap, dt)


def _mixed_matrix(seed):
    """8 processes of 25,000 rows.  Every row has a band of 7 on-process
    columns.  Rows of processes 1-3 also read 2 columns among the last 64 of
    the previous process (halos inside one band of the ghost buffer: narrow
    blocks); rows of processes 4-7 read 8 columns drawn from the whole
    matrix (about 500,000 ghosts in all: wide blocks); process 0 reads
    nothing off-process."""
    rng = np.random.default_rng(seed)
    n_p, per = 8, 25000
    n = n_p * per
    rows = []
    for i in range(n):
        t = i // per
        lo, hi = t * per, (t + 1) * per
        band = np.clip(np.arange(i - 3, i + 4), lo, hi - 1)
        if 1 <= t <= 3:
            extra = lo - 1 - rng.integers(0, 64, size=2)
        elif t >= 4:
            extra = rng.integers(0, n, size=8)
        else:
            extra = np.zeros(0, dtype=np.int64)
        cols = np.concatenate([band, extra])
        rng.shuffle(cols)
        rows.append(cols)
    return _csr_from_rows(n, rows, seed + 1), n_p


@pytest.fixture(scope="module")
def mixed():
    a, n_p = _mixed_matrix(11)
    v = vec_normal(a.n, 12)
    return a, n_p, v, oracle_spmv.spmv_split(a, v, n_p), oracle_spmv.spmv(a, v)


@pytest.mark.parametrize("rcap", [1024, 2048, 4096, 8192])
def test_narrow_and_wide_blocks_f64(mixed, rcap):
    a, n_p, v, split, _ = mixed
    for mode in ("standard", "nap"):
        w = _apply(a, v, n_p, 4, mode, "f64", {"remote_nnz": rcap})
        assert np.array_equal(w, split), (rcap, mode)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_narrow_and_wide_blocks_reduced(mixed, dtype):
    a, n_p, v, _, ref = mixed
    for rcap in (2048, 8192):
        w = _apply(a, v, n_p, 4, "standard", dtype, {"remote_nnz": rcap})
        assert _relerr(w, ref) <= TOL[dtype], rcap


def _packed_and_plain_matrix(seed):
    """8 processes of 196,608 rows (n = 1,572,864).  Every row has its
    diagonal and one neighbour.  Rows of processes 0-3 also read 4 columns
    drawn from the whole matrix: their off-process blocks read ghosts of
    every band densely, each lane group of 16 within a short stretch of the
    ghost buffer (packed words).  In processes 4-7 only every 997th row
    reads 24 columns drawn from the whole matrix (about 2.4 million ghost
    positions), so a block of 1024 rows holds one or two such rows, and with
    two entries per lane (float64) a lane group reads a dozen of them, more
    than 2^19 positions apart (plain int32 positions with slots)."""
    rng = np.random.default_rng(seed)
    n_p, per = 8, 196608
    n = n_p * per
    i = np.arange(n, dtype=np.int64)
    t = i // per
    nb = np.where(i % per == per - 1, i - 1, i + 1)
    far_n = np.where(t < 4, 4, np.where(i % 997 == 0, 24, 0))
    lens = 2 + far_n
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    col = np.empty(int(rowptr[-1]), dtype=np.int64)
    col[rowptr[:-1]] = i
    col[rowptr[:-1] + 1] = nb
    rows_far = np.repeat(i, far_n)
    pos_far = np.repeat(rowptr[:-1] + 2, far_n) + (np.arange(rows_far.size) -
                                                   np.repeat(np.cumsum(far_n) - far_n, far_n))
    col[pos_far] = rng.integers(0, n, size=rows_far.size)
    return CSR(n, rowptr, col.astype(np.int32), vec_normal(int(rowptr[-1]), seed + 1)), n_p


@pytest.fixture(scope="module")
def packed_plain():
    a, n_p = _packed_and_plain_matrix(21)
    v = vec_normal(a.n, 22)
    return a, n_p, v, oracle_spmv.spmv_split(a, v, n_p), oracle_spmv.spmv(a, v)


@pytest.mark.parametrize("rcap", [2048, 8192])
def test_packed_and_plain_blocks(packed_plain, rcap):
    """One plan with packed and plain off-process blocks (float64; float32
    and bfloat16 plans, with 4 and 8 entries per lane, pack more of them):
    float64 w bitwise the oracle's split-order product in both modes,
    float32 and bfloat16 values within tolerance of the float64 oracle."""
    a, n_p, v, split, ref = packed_plain
    for mode, dtype in (("standard", "f64"), ("nap", "f64"), ("standard", "f32"),
                        ("standard", "bf16")):
        vals = {"f64": a.val, "f32": to_f32(a.val), "bf16": bf16_bits(a.val)}[dtype]
        p = nap.Plan(a.rowptr, a.col, vals, a.n, n_p, 4, mode=mode, dtype=dtype)
        p.set_param("remote_nnz", rcap)
        kinds = p.block_kinds()
        assert kinds["packed"] > 0 and (kinds["plain"] > 0 or dtype != "f64"), kinds
        tv = torch.from_numpy(v if dtype == "f64" else to_f32(v)).to(DEV)
        w = torch.full_like(tv, float("nan"))
        p.apply(tv, w)
        torch.cuda.synchronize()
        p.close()
        w = w.cpu().numpy().astype(np.float64)
        if dtype == "f64":
            assert np.array_equal(w, split), (rcap, mode)
        else:
            assert _relerr(w, ref) <= TOL[dtype], (rcap, dtype)
