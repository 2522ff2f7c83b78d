"""A seeded sweep of small random problems through every mode, variant,
partition, value type and tuning, each checked against the oracle: float64
w bitwise against the split-order product (two- or three-part), reduced
precision within tolerance, ghosts bit for bit in the plan's order."""
import numpy as np
import pytest
import torch

import paper_1612_08060_amd as nap
from oracle import spmv as oracle_spmv
from workloads import CSR, bf16_bits, random_pattern, to_f32, vec_normal

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
TOL = {"f32": 1e-5, "bf16": 2e-2}
LAYOUTS = [(1, 1), (2, 1), (2, 2), (6, 2), (8, 4), (12, 3), (16, 8), (20, 4), (32, 16)]
VARIANTS = [(), ("owner_map",), ("split",), ("dedup",), ("three_way",),
            ("owner_map", "dedup", "three_way")]


def _case(i):
    rng = np.random.default_rng(1000 + i)
    n_p, ppn = LAYOUTS[i % len(LAYOUTS)]
    n = int(rng.integers(n_p, 6000))
    a = random_pattern(n, float(rng.uniform(0.0005, 0.02)), seed=2000 + i,
                       empty_rows=int(rng.integers(0, 5)), duplicates=int(rng.integers(0, 5)))
    a = CSR(a.n, a.rowptr, a.col, vec_normal(a.nnz, 3000 + i))
    mode = "standard" if i % 3 == 0 else "nap"
    variant = () if mode == "standard" else VARIANTS[i % len(VARIANTS)]
    strided = i % 5 == 4 and "split" not in variant
    dtype = ("f64", "f64", "f32", "bf16")[i % 4]
    params = {"block_nnz": int(rng.choice([1024, 2048, 4096, 8192])),
              "remote_nnz": int(rng.choice([1024, 2048, 4096, 8192])),
              "window": int(rng.choice([0, 1024, 2048, 4096])),
              "gather_item": int(rng.choice([256, 1000, 65536]))}
    return a, n_p, ppn, mode, variant, strided, dtype, params, vec_normal(n, 4000 + i)


@pytest.mark.parametrize("i", range(48))
def test_sweep(i):
    a, n_p, ppn, mode, variant, strided, dtype, params, v = _case(i)
    print(f"case {i}: n={a.n} nnz={a.nnz} n_p={n_p} ppn={ppn} {mode} {variant} "
          f"strided={strided} {dtype} {params}", flush=True)
    vals = {"f64": a.val, "f32": to_f32(a.val), "bf16": bf16_bits(a.val)}[dtype]
    with nap.Plan(a.rowptr, a.col, vals, a.n, n_p, ppn, mode=mode, dtype=dtype,
                  variant=variant, strided=strided,
                  exchange_copy=(mode == "nap" and i % 2 == 1)) as p:
        for k, x in params.items():
            p.set_param(k, x)
        rows = p.rows()
        x = v if dtype == "f64" else to_f32(v)
        tv = torch.from_numpy(x[rows]).to(DEV)
        w = torch.full_like(tv, float("nan"))
        p.apply(tv, w)
        torch.cuda.synchronize()
        got = np.empty(a.n)
        got[rows] = w.cpu().numpy()
        _, gc = p.ghosts()
        assert np.array_equal(p.read_ghosts(), x[rows][gc])
    if dtype == "f64":
        ref = (oracle_spmv.spmv_split3(a, v, n_p, ppn, strided=strided) if "three_way" in variant
               else oracle_spmv.spmv_split(a, v, n_p, strided=strided))
        assert np.array_equal(got, ref)
    else:
        ref = oracle_spmv.spmv(a, v)
        d = np.linalg.norm(ref)
        assert np.linalg.norm(got - ref) <= TOL[dtype] * (d if d > 0 else 1.0)
