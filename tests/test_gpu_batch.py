"""Caller-owned workspaces, batched applies over many plans, per-partition
applies, HIP graphs and the autotuner, through the C ABI on an MI355X.

Every variant runs the same per-row sums as the plain apply, so every result
must be bitwise equal to the plain apply's (and to the oracle's split-order
product in float64)."""
import os
import tempfile

import numpy as np
import pytest
import torch

import paper_1612_08060_amd as nap
from oracle import spmv as oracle_spmv
from workloads import (bf16_bits, config, kkt_like, laplacian_2d, laplacian_3d, random_pattern,
                       to_f32, vec_normal, vec_uniform)

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _vals(a, dtype):
    return {"f64": a.val, "f32": to_f32(a.val), "bf16": bf16_bits(a.val)}[dtype]


def _plan(a, n_p, ppn, mode="standard", dtype="f64", row_starts=None, **kw):
    return nap.Plan(a.rowptr, a.col, _vals(a, dtype), a.n, n_p, ppn, mode=mode, dtype=dtype,
                    row_starts=row_starts, **kw)


def _vec(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x if dtype == "f64" else to_f32(x))).to(DEV)


def _solo(p, v):
    w = torch.full_like(v, float("nan"))
    p.apply(v, w)
    torch.cuda.synchronize()
    return w


def test_workspaces_concurrent_streams():
    a = kkt_like(1 << 14, 5)
    for mode in ("standard", "nap"):
        p = _plan(a, 32, 8, mode=mode)
        vs = [_vec(vec_normal(a.n, s), "f64") for s in range(4)]
        ref = [_solo(p, v) for v in vs]
        wss = [p.new_workspace() for _ in range(4)]
        outs = [torch.full_like(vs[0], float("nan")) for _ in range(4)]
        streams = [torch.cuda.Stream() for _ in range(4)]
        torch.cuda.synchronize()
        for k in range(4):
            with torch.cuda.stream(streams[k]):
                p.apply_ws(wss[k], vs[k], outs[k], stream=streams[k])
        torch.cuda.synchronize()
        for k in range(4):
            assert torch.equal(outs[k], ref[k]), (mode, k)
            _, gc = p.ghosts()
            assert np.array_equal(p.read_ghosts(ws=wss[k]), vs[k].cpu().numpy()[gc])
        assert p.workspace_bytes >= p.stats["ghosts"] * 8
        p.close()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_batch_mixed_plans_equal_solo(dtype):
    mats = [kkt_like(5000, 1), laplacian_2d(70, 33), laplacian_3d(20, 18, 9),
            random_pattern(300, 0.03, 4, empty_rows=10, duplicates=5), kkt_like(20000, 2)]
    layouts = [(16, 4), (8, 2), (12, 3), (6, 6), (32, 16)]
    plans, vs, refs = [], [], []
    for i, (a, (n_p, ppn)) in enumerate(zip(mats, layouts)):
        mode = "nap" if i % 2 else "standard"
        p = _plan(a, n_p, ppn, mode=mode, dtype=dtype)
        v = _vec(vec_uniform(a.n, 10 + i), dtype)
        plans.append(p)
        vs.append(v)
        refs.append(_solo(p, v))
    # the same matrix twice, with a second workspace
    plans.append(plans[0])
    vs.append(_vec(vec_uniform(mats[0].n, 99), dtype))
    refs.append(_solo(plans[0], vs[-1]))
    wss = [None] * (len(plans) - 1) + [plans[0].new_workspace()]
    b = nap.Batch(16)
    for rep in range(3):
        outs = [torch.full_like(v, float("nan")) for v in vs]
        b.apply(plans, vs, outs, workspaces=wss)
        torch.cuda.synchronize()
        for k, (o, r) in enumerate(zip(outs, refs)):
            assert torch.equal(o, r), (dtype, rep, k)
    if dtype == "f64":
        for k in range(len(mats)):
            ref = oracle_spmv.spmv_split(mats[k], vs[k].cpu().numpy(), layouts[k][0])
            assert np.array_equal(refs[k].cpu().numpy(), ref)
    b.close()
    for p in plans[:-1]:
        p.close()


def test_batch_mixed_remote_block_sizes():
    """Plans with different off-process block sizes in one batch: one second
    launch per size, every product equal to its solo apply bit for bit."""
    a, b2 = kkt_like(1 << 13, 21), laplacian_3d(14, 14, 14)
    plans = []
    for rn, mode in ((1024, "standard"), (8192, "nap"), (2048, "standard"), (4096, "nap"),
                     (8192, "standard"), (1024, "nap")):
        p = _plan(a, 16, 4, mode=mode)
        p.set_param("remote_nnz", rn)
        plans.append(p)
    plans.append(_plan(b2, 8, 4, mode="nap"))
    vs = [_vec(vec_normal(p.n, 30 + k), "f64") for k, p in enumerate(plans)]
    ref = [_solo(p, v) for p, v in zip(plans, vs)]
    outs = [torch.full_like(v, float("nan")) for v in vs]
    bt = nap.Batch(len(plans))
    print("batch of mixed remote block sizes", flush=True)
    bt.apply(plans, vs, outs)
    torch.cuda.synchronize()
    bt.close()
    for k in range(len(plans)):
        assert torch.equal(outs[k], ref[k]), k
    for p in plans:
        p.close()


def test_batch_rejects_mixed_types():
    a = laplacian_2d(16, 16)
    p1 = _plan(a, 4, 2, dtype="f64")
    p2 = _plan(a, 4, 2, dtype="f32")
    b = nap.Batch(4)
    with pytest.raises(nap.NapspmvError):
        b.apply([p1, p2], [_vec(np.ones(a.n), "f64"), _vec(np.ones(a.n), "f32")],
                [torch.zeros(a.n, dtype=torch.float64, device=DEV),
                 torch.zeros(a.n, dtype=torch.float32, device=DEV)])
    p3 = _plan(a, 4, 2, mode="nap", exchange_copy=True)
    with pytest.raises(nap.NapspmvError):
        b.apply([p3], [_vec(np.ones(a.n), "f64")], [torch.zeros(a.n, dtype=torch.float64, device=DEV)])
    with pytest.raises(nap.NapspmvError):
        nap.Batch(0)
    b.close()


def test_partitions_equal_batched():
    wl = config(4, scale=3)                    # 27-point, uneven lognormal blocks
    a = wl.csr
    for dtype in ("f32", "f64"):
        p = _plan(a, wl.n_p, wl.ppn, dtype=dtype, row_starts=wl.row_starts)
        v = _vec(wl.v, dtype)
        ref = _solo(p, v)
        p.prepare_partitions()
        w = torch.full_like(v, float("nan"))
        for t in range(wl.n_p):
            p.apply_partition(t, v, w)
        torch.cuda.synchronize()
        assert torch.equal(w, ref)
        # tuning change rebuilds the per-partition schedules too
        p.set_param("block_nnz", 1024)
        w2 = torch.full_like(v, float("nan"))
        for t in range(wl.n_p):
            p.apply_partition(t, v, w2)
        torch.cuda.synchronize()
        assert torch.equal(w2, ref)
        with pytest.raises(nap.NapspmvError):
            p.apply_partition(wl.n_p, v, w2)
        p.close()
    pn = _plan(a, wl.n_p, wl.ppn, mode="nap", dtype="f32", row_starts=wl.row_starts)
    with pytest.raises(nap.NapspmvError):
        pn.prepare_partitions()
    pn.close()


def test_graph_replays():
    a = kkt_like(1 << 14, 8)
    for mode in ("standard", "nap"):
        p = _plan(a, 32, 8, mode=mode)
        v = _vec(vec_normal(a.n, 3), "f64")
        w = torch.zeros_like(v)
        g = p.graph(v, w)
        for it in range(4):
            w.zero_()
            v.mul_(-1.5)
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(w, _solo(p, v)), (mode, it)
        g.close()
        p.close()


def test_autotune_keeps_results_and_caches():
    a = kkt_like(1 << 15, 13)
    v = _vec(vec_normal(a.n, 14), "f64")
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "tune.txt")
        for mode in ("standard", "nap"):
            p = _plan(a, 64, 16, mode=mode)
            ref = _solo(p, v)
            w = torch.zeros_like(v)
            best = p.autotune(v, w, reps=2, cache_path=cache)
            assert best > 0
            cfg = (p.get_param("block_nnz"), p.get_param("window"), p.get_param("gather_item"),
                   p.get_param("remote_nnz"))
            assert torch.equal(_solo(p, v), ref)
            p.close()
            p2 = _plan(a, 64, 16, mode=mode)
            assert p2.autotune(v, w, reps=2, cache_path=cache) == -1.0      # from the cache
            assert (p2.get_param("block_nnz"), p2.get_param("window"),
                    p2.get_param("gather_item"), p2.get_param("remote_nnz")) == cfg
            assert torch.equal(_solo(p2, v), ref)
            p2.close()
        assert len(open(cache).read().splitlines()) == 2


def test_batched_workload_full_size():
    """The 256-block 27-point workload at full size (N = 2,604,175, 69 M
    entries), in the benchmark's launch configuration: autotuned, the whole
    product as one graph-captured launch pair.  float32 values: w within 1e-5
    of the float64 oracle (normwise), and the per-block launches equal to the
    batched result bit for bit; float64 values: w equal to the oracle's
    split-order product bit for bit."""
    wl = config(4)
    a = wl.csr
    print("batched workload, full size, float32", flush=True)
    p = _plan(a, wl.n_p, wl.ppn, dtype="f32", row_starts=wl.row_starts)
    v = _vec(wl.v, "f32")
    w = torch.full_like(v, float("nan"))
    p.autotune(v, w, reps=2)
    g = p.graph(v, w)
    w.fill_(float("nan"))
    g.launch()
    torch.cuda.synchronize()
    ref = oracle_spmv.spmv(a, wl.v)
    got = w.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= 1e-5, err
    p.prepare_partitions()
    w2 = torch.full_like(v, float("nan"))
    for t in range(wl.n_p):
        p.apply_partition(t, v, w2)
    torch.cuda.synchronize()
    assert torch.equal(w, w2)
    g.close()
    p.close()
    print("batched workload, full size, float64", flush=True)
    p64 = _plan(a, wl.n_p, wl.ppn, dtype="f64", row_starts=wl.row_starts)
    w64 = _solo(p64, _vec(wl.v, "f64"))
    assert np.array_equal(w64.cpu().numpy(), oracle_spmv.spmv_split(a, wl.v, wl.n_p, wl.row_starts))
    p64.close()


def test_batch_mixes_fused_and_separate_nap_scatter():
    """NAP plans that scatter inside the first launch (pack-and-scatter
    items) and NAP plans that keep the separate scatter launch (exchange
    items narrower than a band) in one batch, with standard plans: every
    product equal to its solo apply bit for bit."""
    a, b2 = kkt_like(1 << 13, 41), laplacian_3d(12, 12, 12)
    plans = [_plan(a, 16, 4, mode="nap"), _plan(a, 16, 4, mode="nap"),
             _plan(b2, 8, 4, mode="nap"), _plan(b2, 8, 4, mode="standard")]
    plans[1].set_param("gather_item", 256)
    vs = [_vec(vec_normal(p.n, 60 + k), "f64") for k, p in enumerate(plans)]
    ref = [_solo(p, v) for p, v in zip(plans, vs)]
    for rep in range(2):
        outs = [torch.full_like(v, float("nan")) for v in vs]
        bt = nap.Batch(len(plans))
        print(f"batch of fused and separate NAP scatters, pass {rep}", flush=True)
        bt.apply(plans, vs, outs)
        torch.cuda.synchronize()
        bt.close()
        for k in range(len(plans)):
            assert torch.equal(outs[k], ref[k]), (rep, k)
    for p in plans:
        p.close()
