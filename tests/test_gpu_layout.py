"""Band layout of the exchange buffers on the GPU: re-laying the bands (a new
BLOCK_NNZ) between applies keeps every result bit for bit, in every mode and
through the per-process launches, and ghosts read back in plan order; bands
with no ghost, matrices narrower than one band and a single band all work."""
import numpy as np
import pytest
import torch

import paper_1612_08060_amd as nap
from oracle import spmv as oracle_spmv
from workloads import CSR, kkt_like, random_pattern, vec_normal

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _apply(p, tv):
    w = torch.full_like(tv, float("nan"))
    p.apply(tv, w)
    torch.cuda.synchronize()
    return w.cpu().numpy()


@pytest.mark.parametrize("mode,variant", [("standard", ()), ("nap", ()), ("nap", ("three_way",)),
                                          ("nap", ("split", "owner_map"))])
def test_relayout_between_applies(mode, variant):
    a = kkt_like(3 * 4096 + 517, 21)          # several bands of every width, ragged tail
    v = vec_normal(a.n, 22)
    n_p, ppn = 24, 4
    ref = (oracle_spmv.spmv_split3(a, v, n_p, ppn) if "three_way" in variant
           else oracle_spmv.spmv_split(a, v, n_p))
    tv = torch.from_numpy(v).to(DEV)
    with nap.Plan(a.rowptr, a.col, a.val, a.n, n_p, ppn, mode=mode, variant=variant) as p:
        _, gc = p.ghosts()
        for cap, item, rcap in ((4096, -1, -1), (1024, 300, 1024), (2048, 1 << 20, 4096),
                                (8192, 256, 2048), (4096, 1000, 1024), (-1, -1, -1)):
            print(f"mode={mode} variant={variant} block_nnz={cap} item={item} remote={rcap}", flush=True)
            p.set_param("block_nnz", cap)
            p.set_param("gather_item", item)
            p.set_param("remote_nnz", rcap)
            assert np.array_equal(_apply(p, tv), ref)
            assert np.array_equal(p.read_ghosts(), v[gc])


def test_partitions_follow_relayout():
    a = kkt_like(5000, 23)
    v = vec_normal(a.n, 24)
    n_p = 10
    ref = oracle_spmv.spmv_split(a, v, n_p)
    tv = torch.from_numpy(v).to(DEV)
    with nap.Plan(a.rowptr, a.col, a.val, a.n, n_p, 2, mode="standard") as p:
        p.prepare_partitions()
        for cap, rcap in ((4096, 8192), (1024, 1024), (2048, 4096), (8192, 2048)):
            print(f"partitions block_nnz={cap} remote={rcap}", flush=True)
            p.set_param("block_nnz", cap)
            p.set_param("remote_nnz", rcap)
            w = torch.full_like(tv, float("nan"))
            for t in range(n_p):
                p.apply_partition(t, tv, w)
            torch.cuda.synchronize()
            assert np.array_equal(w.cpu().numpy(), ref)


def test_sparse_bands_and_narrow_matrices():
    """Columns concentrated in a few bands (most bands hold no ghost), a
    matrix narrower than one band, and one with no ghost at all."""
    n = 20000
    rng = np.random.default_rng(7)
    rows = []
    for i in range(n):
        far = rng.integers(0, 300, size=3)              # every far column in band 0
        rows.append(np.unique(np.concatenate([[i], far, [min(n - 1, i + 1)]])))
    rp = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    a = CSR(n, rp, np.concatenate(rows).astype(np.int32), vec_normal(int(rp[-1]), 8))
    v = vec_normal(n, 9)
    tv = torch.from_numpy(v).to(DEV)
    for mode in ("standard", "nap"):
        print(f"sparse bands mode={mode}", flush=True)
        with nap.Plan(a.rowptr, a.col, a.val, a.n, 40, 8, mode=mode) as p:
            assert np.array_equal(_apply(p, tv), oracle_spmv.spmv_split(a, v, 40))
    small = random_pattern(700, 0.02, seed=3, empty_rows=5, duplicates=2)
    small = CSR(small.n, small.rowptr, small.col, vec_normal(small.nnz, 4))
    vs = vec_normal(700, 5)
    ts = torch.from_numpy(vs).to(DEV)
    for mode in ("standard", "nap"):
        for n_p, ppn in ((7, 7), (7, 1), (1, 1), (14, 2)):
            print(f"narrow mode={mode} n_p={n_p} ppn={ppn}", flush=True)
            with nap.Plan(small.rowptr, small.col, small.val, small.n, n_p, ppn, mode=mode) as p:
                assert np.array_equal(_apply(p, ts), oracle_spmv.spmv_split(small, vs, n_p))
                _, gc = p.ghosts()
                assert np.array_equal(p.read_ghosts(), vs[gc])
