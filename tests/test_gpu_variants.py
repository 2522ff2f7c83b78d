"""NAP plan variants on the GPU: the owner mapping, the split of a partner
over several processes and the deduplicated fully local step change the
messages only, so every ghost slot still holds the owner's value bit for bit
and w equals the default plan's (and the oracle's split-order product) bit
for bit."""
import numpy as np
import pytest
import torch

import paper_1612_08060_amd as nap
from oracle import spmv as oracle_spmv
from workloads import CSR, config, random_pattern, vec_normal

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
VARIANTS = [("owner_map",), ("split",), ("dedup",), ("owner_map", "split", "dedup")]


def _apply(a, v, n_p, ppn, variant, row_starts=None, exchange_copy=False):
    with nap.Plan(a.rowptr, a.col, a.val, a.n, n_p, ppn, mode="nap", row_starts=row_starts,
                  variant=variant, exchange_copy=exchange_copy) as p:
        tv = torch.from_numpy(v).to(DEV)
        w = torch.full_like(tv, float("nan"))
        p.apply(tv, w)
        torch.cuda.synchronize()
        g = p.read_ghosts()
        _, gc = p.ghosts()
        return w.cpu().numpy(), g, gc


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("n_p,ppn", [(4, 2), (8, 4), (12, 4), (16, 8)])
def test_random_small(variant, n_p, ppn):
    for seed in range(2):
        n = 80 + 11 * n_p + 5 * seed
        a = random_pattern(n, 0.06, seed=900 + n_p + seed, empty_rows=2, duplicates=3)
        a = CSR(a.n, a.rowptr, a.col, vec_normal(a.nnz, seed))
        v = vec_normal(n, seed + 7)
        print(f"variant={variant} n_p={n_p} ppn={ppn} seed={seed}", flush=True)
        w, g, gc = _apply(a, v, n_p, ppn, variant)
        assert np.array_equal(g, v[gc])
        assert np.array_equal(w, oracle_spmv.spmv_split(a, v, n_p))


@pytest.mark.parametrize("k", [1, 2])
@pytest.mark.parametrize("variant", VARIANTS)
def test_paper_configs(k, variant):
    wl = config(k)
    print(f"config={k} variant={variant}", flush=True)
    w, g, gc = _apply(wl.csr, wl.v, wl.n_p, wl.ppn, variant, wl.row_starts,
                      exchange_copy=(k == 2))
    assert np.array_equal(g, wl.v[gc])
    assert np.array_equal(w, oracle_spmv.spmv_split(wl.csr, wl.v, wl.n_p, wl.row_starts))


def test_kkt_full_all_variants():
    wl = config(3)
    ref = oracle_spmv.spmv_split(wl.csr, wl.v, wl.n_p)
    print("kkt full, all variants", flush=True)
    w, g, gc = _apply(wl.csr, wl.v, wl.n_p, wl.ppn, ("owner_map", "split", "dedup"))
    assert np.array_equal(g, wl.v[gc])
    assert np.array_equal(w, ref)


# -- the three-way product (algorithm NAPSpMV's on_process, on_node, off_node) --

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}


def _vals(a, dtype):
    from workloads import bf16_bits, to_f32
    return {"f64": a.val, "f32": to_f32(a.val), "bf16": bf16_bits(a.val)}[dtype]


@pytest.mark.parametrize("n_p,ppn", [(1, 1), (4, 1), (4, 4), (8, 4), (12, 3), (16, 8)])
def test_three_way_random_small(n_p, ppn):
    for seed in range(2):
        n = 90 + 7 * n_p + 3 * seed
        a = random_pattern(n, 0.07, seed=300 + n_p + seed, empty_rows=2, duplicates=3)
        a = CSR(a.n, a.rowptr, a.col, vec_normal(a.nnz, seed + 1))
        v = vec_normal(n, seed + 9)
        print(f"three_way n_p={n_p} ppn={ppn} seed={seed}", flush=True)
        for copy in (False, True):
            w, g, gc = _apply(a, v, n_p, ppn, ("three_way",), exchange_copy=copy)
            assert np.array_equal(g, v[gc])
            assert np.array_equal(w, oracle_spmv.spmv_split3(a, v, n_p, ppn))


@pytest.mark.parametrize("k", [1, 2, 4])
def test_three_way_paper_configs(k):
    wl = config(k)
    a = wl.csr
    print(f"three_way config={k}", flush=True)
    if k == 4:      # float32 values: compare with the float64 oracle of the same values
        with nap.Plan(a.rowptr, a.col, _vals(a, "f32"), a.n, wl.n_p, wl.ppn, mode="nap",
                      dtype="f32", row_starts=wl.row_starts, variant=("three_way",)) as p:
            tv = torch.from_numpy(wl.v.astype(np.float32)).to(DEV)
            w = torch.full_like(tv, float("nan"))
            p.apply(tv, w)
            torch.cuda.synchronize()
            ref = oracle_spmv.spmv(a, wl.v)
            err = np.linalg.norm(w.cpu().numpy() - ref) / np.linalg.norm(ref)
            assert err <= TOL["f32"], err
        return
    w, g, gc = _apply(a, wl.v, wl.n_p, wl.ppn, ("three_way",), wl.row_starts)
    assert np.array_equal(g, wl.v[gc])
    assert np.array_equal(w, oracle_spmv.spmv_split3(a, wl.v, wl.n_p, wl.ppn, wl.row_starts))


@pytest.fixture(scope="module")
def kkt():
    wl = config(3)
    return wl, oracle_spmv.spmv(wl.csr, wl.v), oracle_spmv.spmv_split3(wl.csr, wl.v, wl.n_p, wl.ppn)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_three_way_kkt_full(kkt, dtype):
    wl, ref, split3 = kkt
    a = wl.csr
    print(f"three_way kkt dtype={dtype}", flush=True)
    with nap.Plan(a.rowptr, a.col, _vals(a, dtype), a.n, wl.n_p, wl.ppn, mode="nap",
                  dtype=dtype, variant=("three_way",)) as p:
        x = wl.v if dtype == "f64" else wl.v.astype(np.float32)
        tv = torch.from_numpy(x).to(DEV)
        w = torch.full_like(tv, float("nan"))
        p.apply(tv, w)
        torch.cuda.synchronize()
        got = w.cpu().numpy().astype(np.float64)
    if dtype == "f64":
        assert np.array_equal(got, split3)
        rows = np.random.default_rng(1).choice(a.n, 48, replace=False)
        assert np.array_equal(got[rows],
                              oracle_spmv.spmv_split3_rows(a, wl.v, wl.n_p, wl.ppn, rows))
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err <= TOL[dtype], err


def test_three_way_stages_streams_graph_server():
    """Per-stage launches on a side stream, graph replays with eager work
    between them, and a server (which runs such plans alone) all give the
    three-way result bit for bit; batches refuse the plan."""
    wl = config(2)
    a = wl.csr
    ref = oracle_spmv.spmv_split3(a, wl.v, wl.n_p, wl.ppn)
    with nap.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="nap",
                  variant=("three_way",)) as p:
        tv = torch.from_numpy(wl.v).to(DEV)
        w = torch.full_like(tv, float("nan"))
        side = torch.cuda.Stream()
        print("three_way stages on a side stream", flush=True)
        p.apply_stage(nap.STAGE_LOCAL, tv, w, stream=side)
        p.apply_stage(nap.STAGE_REMOTE, tv, w, stream=side)
        side.synchronize()
        assert np.array_equal(w.cpu().numpy(), ref)
        print("three_way graph replays", flush=True)
        wg = torch.full_like(tv, float("nan"))
        g = p.graph(tv, wg)
        for r in range(3):
            wg.fill_(float("nan"))
            g.launch()
            torch.cuda.synchronize()
            assert np.array_equal(wg.cpu().numpy(), ref), r
            w2 = torch.full_like(tv, float("nan"))
            p.apply(tv, w2)                     # eager work between replays
            torch.cuda.synchronize()
            assert np.array_equal(w2.cpu().numpy(), ref)
        g.close()
        print("three_way batch refused", flush=True)
        b = nap.Batch(2)
        with pytest.raises(nap.NapspmvError) as e:
            b.apply([p, p], [tv, tv], [w, wg])
        assert e.value.code == -4
        b.close()
        print("three_way server", flush=True)
        srv = nap.Server(slots=2, max_batch=8)
        pid = srv.add(p)
        outs = [torch.full_like(tv, float("nan")) for _ in range(4)]
        tickets = [srv.submit(pid, tv, o) for o in outs]
        for t in tickets:
            srv.wait(t)
        torch.cuda.synchronize()
        for o in outs:
            assert np.array_equal(o.cpu().numpy(), ref)
        srv.close()
