"""Strided partition on the GPU: v and w in process-major order (position k
holds row rows[k]); ghosts hold the owners' values bit for bit, and float64 w
equals the oracle's split-order product under the strided owner map bit for
bit (two-way for standard and default NAP plans, three-way for three_way)."""
import numpy as np
import pytest
import torch

import paper_1612_08060_amd as nap
from oracle import spmv as oracle_spmv
from workloads import CSR, config, random_pattern, to_f32, vec_normal

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _apply(a, v, n_p, ppn, mode, variant=(), dtype="f64", vals=None):
    with nap.Plan(a.rowptr, a.col, a.val if vals is None else vals, a.n, n_p, ppn, mode=mode,
                  dtype=dtype, variant=variant, strided=True) as p:
        rows = p.rows()
        x = v[rows] if dtype == "f64" else to_f32(v)[rows]
        tv = torch.from_numpy(x).to(DEV)
        w = torch.full_like(tv, float("nan"))
        p.apply(tv, w)
        torch.cuda.synchronize()
        g = p.read_ghosts()
        _, gc = p.ghosts()
        out = np.empty(a.n)
        out[rows] = w.cpu().numpy()
        # ghost columns are positions: map back to rows
        return out, g, rows[gc]


@pytest.mark.parametrize("n_p,ppn", [(1, 1), (4, 2), (6, 3), (16, 4)])
@pytest.mark.parametrize("mode,variant", [("standard", ()), ("nap", ()), ("nap", ("three_way",)),
                                          ("nap", ("owner_map", "dedup"))])
def test_random_small(n_p, ppn, mode, variant):
    for seed in range(2):
        n = 70 + 9 * n_p + seed
        a = random_pattern(n, 0.07, seed=600 + n_p + seed, empty_rows=2, duplicates=2)
        a = CSR(a.n, a.rowptr, a.col, vec_normal(a.nnz, seed + 2))
        v = vec_normal(n, seed + 5)
        print(f"strided n_p={n_p} ppn={ppn} mode={mode} variant={variant} seed={seed}", flush=True)
        w, g, gcol = _apply(a, v, n_p, ppn, mode, variant)
        assert np.array_equal(g, v[gcol])
        ref = (oracle_spmv.spmv_split3(a, v, n_p, ppn, strided=True) if "three_way" in variant
               else oracle_spmv.spmv_split(a, v, n_p, strided=True))
        assert np.array_equal(w, ref)


@pytest.mark.parametrize("mode", ["standard", "nap"])
def test_kkt_full(mode):
    wl = config(3)
    a = wl.csr
    print(f"strided kkt mode={mode}", flush=True)
    w, g, gcol = _apply(a, wl.v, wl.n_p, wl.ppn, mode)
    assert np.array_equal(g, wl.v[gcol])
    assert np.array_equal(w, oracle_spmv.spmv_split(a, wl.v, wl.n_p, strided=True))


def test_laplace3d_f32():
    wl = config(2)
    a = wl.csr
    print("strided laplace3d f32", flush=True)
    w, g, gcol = _apply(a, wl.v, wl.n_p, wl.ppn, "nap", dtype="f32", vals=to_f32(a.val))
    assert np.array_equal(g, to_f32(wl.v)[gcol])
    ref = oracle_spmv.spmv(a, wl.v)
    assert np.linalg.norm(w - ref) / np.linalg.norm(ref) <= 1e-5


def test_strided_partitions_and_batch():
    """Per-process launches and a batch of a strided plan give the plan's own
    result bit for bit."""
    a = random_pattern(3000, 0.01, seed=77, duplicates=2)
    a = CSR(a.n, a.rowptr, a.col, vec_normal(a.nnz, 78))
    v = vec_normal(a.n, 79)
    with nap.Plan(a.rowptr, a.col, a.val, a.n, 12, 4, mode="standard", strided=True) as p:
        rows = p.rows()
        tv = torch.from_numpy(v[rows]).to(DEV)
        w0 = torch.full_like(tv, float("nan"))
        p.apply(tv, w0)
        p.prepare_partitions()
        w1 = torch.full_like(tv, float("nan"))
        for t in range(12):
            p.apply_partition(t, tv, w1)
        b = nap.Batch(2)
        ws2 = p.new_workspace()
        w2 = torch.full_like(tv, float("nan"))
        w3 = torch.full_like(tv, float("nan"))
        b.apply([p, p], [tv, tv], [w2, w3], workspaces=[None, ws2])
        torch.cuda.synchronize()
        b.close()
        out = np.empty(a.n)
        out[rows] = w0.cpu().numpy()
        assert np.array_equal(out, oracle_spmv.spmv_split(a, v, 12, strided=True))
        for w in (w1, w2, w3):
            assert torch.equal(w, w0)
