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
