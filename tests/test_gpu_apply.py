"""Parity of the HIP path with the oracle, through the C ABI, on an MI355X.

* ghost buffers: after the exchange every ghost slot holds the owner's value,
  bit for bit (both communication modes);
* w: float64 plans sum every row as algorithm standard_spmv does (on-process
  entries, then off-process entries, each in stored order, one rounded
  product and one rounded add per entry), so w is bitwise equal to the
  oracle's split-order product, and within 1e-12 normwise of the plain
  product; standard and NAP results are bitwise identical, for every tuning;
* reduced precision: float32 values within 1e-5 and bfloat16 values within
  2e-2 normwise of the float64 oracle (float32 accumulation);
* edge cases: one process, one node, one process per node, remainder rows,
  explicit uneven blocks, empty rows, duplicate entries, a matrix with no
  entries, the explicit exchange copy, per-stage launches, non-default
  streams, graph capture and replay, the device-memory budget.
"""
import numpy as np
import pytest
import torch

import paper_1612_08060_amd as nap
from oracle import brute, spmv as oracle_spmv
from tests.helpers import example_2_1
from workloads import (CSR, bf16_bits, bf16_to_f32, config, kkt_like, laplacian_2d,
                       random_pattern, to_f32, vec_normal, vec_uniform)

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}


def _vals(a, dtype):
    return {"f64": a.val, "f32": to_f32(a.val), "bf16": bf16_bits(a.val)}[dtype]


def _run(a, v, n_p, ppn, mode, dtype="f64", row_starts=None, params=None, **kw):
    """Apply through the library; returns (w as float64 numpy, ghost values, ghost cols)."""
    p = nap.Plan(a.rowptr, a.col, _vals(a, dtype), a.n, n_p, ppn, mode=mode, dtype=dtype,
                 row_starts=row_starts, **kw)
    for k, x in (params or {}).items():
        p.set_param(k, x)
    tv = torch.from_numpy(v if dtype == "f64" else to_f32(v)).to(DEV)
    w = torch.full_like(tv, float("nan"))
    p.apply(tv, w)
    torch.cuda.synchronize()
    g = p.read_ghosts()
    _, gc = p.ghosts()
    p.close()
    return w.cpu().numpy().astype(np.float64), g, gc


def _relerr(w, ref):
    d = np.linalg.norm(ref)
    return np.linalg.norm(w - ref) / (d if d > 0 else 1.0)


def _split(a, v, n_p, row_starts=None):
    return oracle_spmv.spmv_split(a, v, n_p, row_starts)


def _check_ghosts(g, gc, v, dtype):
    expect = v[gc] if dtype == "f64" else to_f32(v)[gc]
    assert np.array_equal(g, expect)


@pytest.mark.parametrize("mode", ["standard", "nap"])
def test_example_2_1_exact(mode):
    _, a = example_2_1()
    a = CSR(a.n, a.rowptr, a.col, np.arange(1, a.nnz + 1, dtype=np.float64))
    v = np.array([3.0, -1.0, 4.0, 1.0, -5.0, 9.0])
    w, g, gc = _run(a, v, 6, 2, mode)
    _check_ghosts(g, gc, v, "f64")
    assert np.array_equal(w, brute.matvec(a, v))


@pytest.mark.parametrize("n_p,ppn", [(1, 1), (4, 1), (4, 4), (6, 2), (8, 4), (12, 3), (48, 4)])
def test_random_small(n_p, ppn):
    for seed in range(2):
        n = 50 * (seed + 1) + 3 * n_p + 1
        a = random_pattern(n, 0.08, seed=seed + n_p, empty_rows=3, duplicates=4)
        a = CSR(a.n, a.rowptr, a.col, vec_normal(a.nnz, seed))
        v = vec_normal(n, seed + 100)
        ref = _split(a, v, n_p)
        res = {}
        for mode in ("standard", "nap"):
            w, g, gc = _run(a, v, n_p, ppn, mode)
            _check_ghosts(g, gc, v, "f64")
            assert np.array_equal(w, ref)
            assert _relerr(w, oracle_spmv.spmv(a, v)) <= TOL["f64"]
            res[mode] = w
        assert np.array_equal(res["standard"], res["nap"])


def test_laplace2d_exact_and_constant():
    wl = config(1)
    a = wl.csr
    v_int = ((np.arange(a.n) % 7) - 3).astype(np.float64)
    ref = oracle_spmv.spmv(a, v_int)
    for mode in ("standard", "nap"):
        w, g, gc = _run(a, v_int, wl.n_p, wl.ppn, mode)
        assert np.array_equal(w, ref)
        w1, _, _ = _run(a, np.ones(a.n), wl.n_p, wl.ppn, mode)
        x, y = np.arange(a.n) % 64, np.arange(a.n) // 64
        interior = (x > 0) & (x < 63) & (y > 0) & (y < 63)
        assert np.all(w1[interior] == 0.0) and np.all(w1[~interior] > 0)
        w, g, gc = _run(a, wl.v, wl.n_p, wl.ppn, mode)
        _check_ghosts(g, gc, wl.v, "f64")
        assert _relerr(w, oracle_spmv.spmv(a, wl.v)) <= TOL["f64"]


@pytest.fixture(scope="module")
def laplace3d():
    return config(2)


@pytest.mark.parametrize("mode", ["standard", "nap"])
def test_laplace3d_full(laplace3d, mode):
    wl = laplace3d
    w, g, gc = _run(wl.csr, wl.v, wl.n_p, wl.ppn, mode)
    _check_ghosts(g, gc, wl.v, "f64")
    assert np.array_equal(w, _split(wl.csr, wl.v, wl.n_p))
    assert _relerr(w, oracle_spmv.spmv(wl.csr, wl.v)) <= TOL["f64"]


def test_laplace3d_modes_bitwise(laplace3d):
    wl = laplace3d
    ws, _, _ = _run(wl.csr, wl.v, wl.n_p, wl.ppn, "standard")
    wn, _, _ = _run(wl.csr, wl.v, wl.n_p, wl.ppn, "nap", exchange_copy=True)
    assert np.array_equal(ws, wn)


@pytest.fixture(scope="module")
def kkt():
    wl = config(3)
    ref = oracle_spmv.spmv(wl.csr, wl.v)
    split = _split(wl.csr, wl.v, wl.n_p)
    return wl, ref, split


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_kkt_full_dtypes(kkt, dtype):
    wl, ref, split = kkt
    w, g, gc = _run(wl.csr, wl.v, wl.n_p, wl.ppn, "standard", dtype=dtype)
    _check_ghosts(g, gc, wl.v, dtype)
    err = _relerr(w, ref)
    assert err <= TOL[dtype], err
    if dtype == "f64":
        assert np.array_equal(w, split)
    # sampled rows computed one by one by the oracle
    rows = np.random.default_rng(0).choice(wl.csr.n, 64, replace=False)
    s = oracle_spmv.spmv_split_rows(wl.csr, wl.v, wl.n_p, rows)
    if dtype == "f64":
        assert np.array_equal(w[rows], s)
    assert np.allclose(w[rows], s, rtol=0, atol=TOL[dtype] * 50 * np.abs(s).max())


def test_kkt_full_nap_bitwise(kkt):
    wl, ref, split = kkt
    ws, _, _ = _run(wl.csr, wl.v, wl.n_p, wl.ppn, "standard")
    wn, g, gc = _run(wl.csr, wl.v, wl.n_p, wl.ppn, "nap")
    _check_ghosts(g, gc, wl.v, "f64")
    assert np.array_equal(ws, wn)


@pytest.mark.parametrize("block_nnz,item,window,remote", [(1024, 256, 0, 1024), (2048, 3000, 1024, 8192),
                                                          (4096, 65536, 4096, 2048), (-1, -1, -1, -1),
                                                          (2048, 1 << 20, 2048, 4096),
                                                          (8192, 777, 4096, 8192), (8192, 4096, 0, 1024)])
def test_stream_schedules_bitwise(block_nnz, item, window, remote):
    a = kkt_like(1 << 15, 11)
    v = vec_normal(a.n, 12)
    ref = _split(a, v, 64)
    for mode in ("standard", "nap"):
        w, g, gc = _run(a, v, 64, 16, mode, params={"block_nnz": block_nnz, "gather_item": item,
                                                    "window": window, "remote_nnz": remote})
        _check_ghosts(g, gc, v, "f64")
        assert np.array_equal(w, ref)


def test_long_rows():
    """Rows longer than a stream block are walked in order, chunk by chunk."""
    n = 3000
    rng = np.random.default_rng(5)
    rows = [np.sort(rng.choice(n, size=(2999 if i in (7, 1500) else 1 + i % 9), replace=False))
            for i in range(n)]
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    a = CSR(n, rp, np.concatenate(rows).astype(np.int32), rng.standard_normal(int(rp[-1])))
    v = vec_normal(n, 6)
    ref = _split(a, v, 12)
    for bn in (1024, 2048, 4096):
        for win in (0, 1024, 4096):
            w, _, _ = _run(a, v, 12, 4, "nap", params={"block_nnz": bn, "window": win})
            assert np.array_equal(w, ref), (bn, win)
    for dtype in ("f32", "bf16"):
        w, _, _ = _run(a, v, 12, 4, "standard", dtype=dtype)
        assert _relerr(w, oracle_spmv.spmv(a, v)) <= TOL[dtype]


@pytest.mark.parametrize("block_nnz", [1024, 2048, 4096])
def test_reduced_precision_schedules(block_nnz):
    a = kkt_like(1 << 15, 21)
    v = vec_normal(a.n, 22)
    ref = oracle_spmv.spmv(a, v)
    for dtype in ("f32", "bf16"):
        for mode in ("standard", "nap"):
            w, g, gc = _run(a, v, 64, 16, mode, dtype=dtype,
                            params={"block_nnz": block_nnz, "window": 1024})
            _check_ghosts(g, gc, v, dtype)
            assert _relerr(w, ref) <= TOL[dtype], (block_nnz, dtype)


def test_bf16_exact_on_laplacian_integers():
    """4, -1 and small integers are exact in bfloat16 and float32 sums."""
    wl = config(1)
    v = ((np.arange(wl.csr.n) % 7) - 3).astype(np.float64)
    ref = oracle_spmv.spmv(wl.csr, v)
    for dtype in ("f32", "bf16"):
        w, _, _ = _run(wl.csr, v, wl.n_p, wl.ppn, "nap", dtype=dtype)
        assert np.array_equal(w, ref)


@pytest.mark.parametrize("window", [0, 1024, 4096])
def test_window_on_small_and_banded(window):
    """Windows wider than the matrix, and windows that cover only part of a
    block's on-process columns (a wide band), give the oracle's w exactly."""
    for n, band in ((300, 40), (20000, 3000)):
        a = kkt_like(n, 7, band=band)
        v = vec_normal(n, 8)
        for n_p, ppn in ((1, 1), (4, 2)):
            w, _, _ = _run(a, v, n_p, ppn, "standard", params={"window": window})
            assert np.array_equal(w, _split(a, v, n_p)), (n, n_p, window)
        w, _, _ = _run(a, v, 4, 2, "standard", dtype="f32", params={"window": window})
        assert _relerr(w, oracle_spmv.spmv(a, v)) <= TOL["f32"]


def test_uneven_blocks_f32():
    wl = config(4, scale=3)
    ref = oracle_spmv.spmv(wl.csr, wl.v)
    for mode in ("standard", "nap"):
        w, g, gc = _run(wl.csr, wl.v, wl.n_p, wl.ppn, mode, dtype="f32",
                        row_starts=wl.row_starts)
        w64, _, _ = _run(wl.csr, wl.v, wl.n_p, wl.ppn, mode, row_starts=wl.row_starts)
        assert np.array_equal(w64, _split(wl.csr, wl.v, wl.n_p, wl.row_starts))
        _check_ghosts(g, gc, wl.v, "f32")
        assert _relerr(w, ref) <= TOL["f32"]


def test_remainder_rows_and_empty_matrix():
    a = random_pattern(203, 0.03, seed=5, empty_rows=20)
    v = vec_uniform(203, 6)
    for mode in ("standard", "nap"):
        w, _, _ = _run(a, v, 16, 4, mode)          # 203 = 16 * 12 + 11
        assert np.array_equal(w, _split(a, v, 16))
    e = CSR(64, np.zeros(65, np.int64), np.zeros(0, np.int32), np.zeros(0))
    w, g, _ = _run(e, vec_uniform(64, 1), 8, 2, "nap")
    assert np.array_equal(w, np.zeros(64)) and g.size == 0


def _saddle(n1, m, seed):
    """[[H, B^T], [B, 0]]: H banded n1 x n1, B m x n1 with 4 random columns
    per row, a zero m x m block; rows store ascending columns."""
    rng = np.random.default_rng(seed)
    rows = [set(range(max(0, i - 2), min(n1, i + 3))) for i in range(n1)] + [set() for _ in range(m)]
    for q in range(m):
        for j in rng.integers(0, n1, 4):
            rows[n1 + q].add(int(j))
            rows[int(j)].add(n1 + q)
    rp = np.zeros(n1 + m + 1, np.int64)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate([np.array(sorted(r), np.int32) for r in rows])
    return CSR(n1 + m, rp, col, vec_normal(col.size, seed + 1))


@pytest.mark.parametrize("block_nnz", [1024, 4096])
def test_saddle_point_zero_block_at_process_boundary(block_nnz):
    """The B rows form whole processes and own no column they use, so their
    on-process row blocks are empty; their clamped loads must not reach past
    v (16-bit columns are offsets from the block's own process)."""
    a = _saddle(3000, 1000, 8)
    starts = np.array([0, 1000, 2000, 3000, 4000], np.int64)
    v = vec_normal(a.n, 9)
    ref = _split(a, v, 4, starts)
    for mode in ("standard", "nap"):
        for dtype in ("f64", "f32", "bf16"):
            w, g, gc = _run(a, v, 4, 2, mode, dtype=dtype, row_starts=starts,
                            params={"block_nnz": block_nnz})
            _check_ghosts(g, gc, v, dtype)
            if dtype == "f64":
                assert np.array_equal(w, ref), mode
            else:
                assert _relerr(w, oracle_spmv.spmv(a, v)) <= TOL[dtype], (mode, dtype)


def test_stages_streams_and_graph():
    a = kkt_like(1 << 14, 3)
    v = torch.from_numpy(vec_normal(a.n, 4)).to(DEV)
    ref = oracle_spmv.spmv(a, v.cpu().numpy())
    p = nap.Plan(a.rowptr, a.col, a.val, a.n, 32, 8, mode="nap", exchange_copy=True)
    w0 = torch.empty_like(v)
    p.apply(v, w0)
    torch.cuda.synchronize()
    assert _relerr(w0.cpu().numpy(), ref) <= TOL["f64"]
    s = torch.cuda.Stream()
    w1 = torch.zeros_like(v)
    with torch.cuda.stream(s):
        p.apply_stage(nap.STAGE_LOCAL, v, w1, stream=s)
        p.apply_stage(nap.STAGE_REMOTE, v, w1, stream=s)
    s.synchronize()
    assert torch.equal(w0, w1)
    # capture one apply in a graph; replay with eager work in between
    w2 = torch.zeros_like(v)
    g = torch.cuda.CUDAGraph()
    cs = torch.cuda.Stream()
    with torch.cuda.stream(cs):
        with torch.cuda.graph(g, stream=cs):
            p.apply(v, w2, stream=cs)
    for it in range(4):
        w2.zero_()
        v.mul_(2.0)
        g.replay()
        torch.cuda.synchronize()
        expect = torch.empty_like(v)
        p.apply(v, expect)
        torch.cuda.synchronize()
        assert torch.equal(w2, expect), it
    p.close()


def test_device_budget():
    a = laplacian_2d(32, 32)
    nap.set_device_budget(1024)
    try:
        with pytest.raises(nap.NapspmvError) as e:
            nap.Plan(a.rowptr, a.col, a.val, a.n, 4, 2)
        assert e.value.code == -2
    finally:
        nap.set_device_budget(0)
    before = nap.device_bytes_in_use()
    p = nap.Plan(a.rowptr, a.col, a.val, a.n, 4, 2)
    assert nap.device_bytes_in_use() - before == p.stats["device_bytes"] > 0
    p.close()
    assert nap.device_bytes_in_use() == before


def test_apply_argument_checks():
    a = laplacian_2d(16, 16)
    p = nap.Plan(a.rowptr, a.col, a.val, a.n, 4, 2)
    v = torch.zeros(a.n, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        p.apply(v, torch.zeros(a.n, dtype=torch.float32, device=DEV))
    with pytest.raises(nap.NapspmvError):
        p.apply(v, v)                               # overlapping input and output
    with pytest.raises(nap.NapspmvError):
        p.apply_stage(7, v, torch.zeros_like(v))
    p.close()


def test_nap_scatter_inside_first_launch():
    """A NAP plan that receives in place packs and scatters band by band in
    the first launch: after STAGE_LOCAL alone every ghost already holds its
    owner's value, and STAGE_REMOTE then completes w.  With exchange items
    narrower than a band (no fusing) or the explicit hop, the scatter stays
    in STAGE_REMOTE; every form gives the same w bit for bit."""
    wl = config(2)
    a = wl.csr
    ref = _split(a, wl.v, wl.n_p, wl.row_starts)
    tv = torch.from_numpy(wl.v).to(DEV)
    for kw, item in (({}, -1), ({}, 256), ({"exchange_copy": True}, -1)):
        print(f"nap stages {kw} gather_item={item}", flush=True)
        with nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="nap",
                      row_starts=wl.row_starts, **kw) as p:
            p.set_param("gather_item", item)
            w = torch.full_like(tv, float("nan"))
            p.apply_stage(nap.STAGE_LOCAL, tv, w)
            torch.cuda.synchronize()
            _, gc = p.ghosts()
            if not kw and item == -1:
                assert np.array_equal(p.read_ghosts(), wl.v[gc])
            p.apply_stage(nap.STAGE_REMOTE, tv, w)
            torch.cuda.synchronize()
            assert np.array_equal(w.cpu().numpy(), ref)
            assert np.array_equal(p.read_ghosts(), wl.v[gc])
