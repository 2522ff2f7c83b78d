"""The serving engine (napspmv_server_*) on an MI355X: many resident plans of
mixed value types and modes, requests admitted into slots as slots and
workspace memory free up, batched per kernel group.  Every request's result
must be bitwise the result of the same apply done alone, and must match the
oracle: float64 bitwise its split-order product (algorithm standard_spmv's
row sums), float32 values within 1e-5 and bfloat16 values within 2e-2
normwise of the float64 product."""
import numpy as np
import pytest
import torch

import paper_1612_08060_amd as nap
from oracle import spmv as oracle_spmv
from workloads import (bf16_bits, kkt_like, laplacian_2d, laplacian_3d, poisson_arrivals,
                       random_pattern, stencil_27, to_f32, vec_uniform)

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _mats():
    specs = [(kkt_like(6000, 3), 16, 4, "standard", "f64"),
             (laplacian_2d(90, 40), 8, 4, "nap", "f64"),
             (laplacian_3d(24, 20, 10), 16, 16, "standard", "f32"),
             (stencil_27(20000), 32, 16, "nap", "f32"),
             (kkt_like(9000, 4), 48, 16, "nap", "bf16"),
             (random_pattern(400, 0.02, 6, empty_rows=4), 4, 2, "standard", "bf16"),
             (laplacian_2d(64, 64), 16, 4, "standard", "f64"),
             (kkt_like(30000, 5), 64, 16, "standard", "f32")]
    out = []
    for a, n_p, ppn, mode, dt in specs:
        val = {"f64": a.val, "f32": to_f32(a.val), "bf16": bf16_bits(a.val)}[dt]
        out.append((a, nap.Plan(a.rowptr, a.col, val, a.n, n_p, ppn, mode=mode, dtype=dt), dt))
    return out


TOL = {"f32": 1e-5, "bf16": 2e-2}


def _check_oracle(a, n_p, dt, v64, got):
    """One served result against the oracle (float64 A and v)."""
    w = got.cpu().numpy().astype(np.float64)
    if dt == "f64":
        assert np.array_equal(w, oracle_spmv.spmv_split(a, v64, n_p))
    else:
        ref = oracle_spmv.spmv(a, v64)
        assert np.linalg.norm(w - ref) / max(np.linalg.norm(ref), 1e-300) <= TOL[dt]


def _vec(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x if dt == "f64" else to_f32(x))).to(DEV)


def _requests(mats, n, seed):
    """(matrix ids, device vectors, the float64 host vectors they came from)."""
    rng = np.random.default_rng(seed)
    ids = rng.integers(0, len(mats), size=n)
    v64 = [vec_uniform(mats[i][0].n, 100 + k) for k, i in enumerate(ids)]
    return ids, [_vec(x, mats[i][2]) for x, i in zip(v64, ids)], v64


def _solo(mats, ids, vs):
    out = []
    for i, v in zip(ids, vs):
        w = torch.empty_like(v)
        mats[i][1].apply(v, w)
        out.append(w)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("slots,max_batch,budget", [(2, 8, 0), (4, 3, 0), (1, 1, 0),
                                                    (3, 6, 2 << 20)])
def test_submit_poll_matches_solo(slots, max_batch, budget):
    mats = _mats()
    ids, vs, v64 = _requests(mats, 60, seed=slots * 10 + max_batch)
    ref = _solo(mats, ids, vs)
    srv = nap.Server(slots=slots, max_batch=max_batch, workspace_budget=budget)
    pids = [srv.add(p) for _, p, _ in mats]
    outs = [torch.full_like(v, float("nan")) for v in vs]
    tickets = [srv.submit(pids[i], v, w) for i, v, w in zip(ids, vs, outs)]
    srv.wait(tickets[-1])
    for t in tickets:
        srv.wait(t)
    torch.cuda.synchronize()
    sizes = []
    for k, t in enumerate(tickets):
        sub, done, bs = srv.info(t)
        assert done >= sub and 1 <= bs <= max_batch
        sizes.append(bs)
        assert torch.equal(outs[k], ref[k]), k
        a, p, dt = mats[ids[k]]
        _check_oracle(a, p.n_p, dt, v64[k], outs[k])
    if max_batch > 1:
        assert max(sizes) > 1                 # requests were batched
    if budget:
        assert srv.workspace_bytes <= budget
    srv.close()
    for _, p, _ in mats:
        p.close()


def test_replay_trace_matches_solo():
    mats = _mats()
    srv = nap.Server(slots=4, max_batch=8)
    pids = [srv.add(p) for _, p, _ in mats]
    ids, arrival = poisson_arrivals(200, 20000.0, len(mats), seed=9)
    v64 = [vec_uniform(mats[i][0].n, 500 + k) for k, i in enumerate(ids)]
    vs = [_vec(x, mats[i][2]) for x, i in zip(v64, ids)]
    ref = _solo(mats, ids, vs)
    outs = [torch.full_like(v, float("nan")) for v in vs]
    lat, bs = srv.replay([pids[i] for i in ids], arrival, vs, outs)
    torch.cuda.synchronize()
    assert np.all(lat > 0) and np.all(bs >= 1)
    for k in range(len(ids)):
        assert torch.equal(outs[k], ref[k]), k
        a, p, dt = mats[ids[k]]
        _check_oracle(a, p.n_p, dt, v64[k], outs[k])
    srv.close()
    for _, p, _ in mats:
        p.close()


def test_server_rejects_bad_arguments():
    with pytest.raises(nap.NapspmvError):
        nap.Server(slots=0)
    srv = nap.Server(slots=1, max_batch=1)
    with pytest.raises(nap.NapspmvError):
        srv.wait(5)
    srv.close()


def test_mixed_kernel_groups_and_solo_plans():
    """Plans that differ in REMOTE_NNZ share a kernel group (one second
    launch per block size), plans that differ in BLOCK_NNZ do not; an
    explicit-hop NAP plan, a three-way plan and a strided plan run alone or
    in their groups; every result equals the apply done alone and, bit for
    bit, the oracle's product in the plan's summation order (the three-way
    plan's is algorithm NAPSpMV's; the strided plan works in process-major
    order)."""
    a1, a2, a3 = kkt_like(7000, 11), kkt_like(5000, 12), laplacian_2d(70, 50)
    plans = [nap.Plan(a1.rowptr, a1.col, a1.val, a1.n, 16, 4, mode="standard"),
             nap.Plan(a1.rowptr, a1.col, a1.val, a1.n, 16, 4, mode="standard"),
             nap.Plan(a2.rowptr, a2.col, a2.val, a2.n, 20, 4, mode="nap", exchange_copy=True),
             nap.Plan(a2.rowptr, a2.col, a2.val, a2.n, 20, 4, mode="nap", variant=("three_way",)),
             nap.Plan(a3.rowptr, a3.col, a3.val, a3.n, 14, 7, mode="nap", strided=True),
             nap.Plan(a3.rowptr, a3.col, a3.val, a3.n, 14, 7, mode="nap",
                      variant=("owner_map", "dedup"))]
    plans[1].set_param("remote_nnz", 2048)
    plans[5].set_param("block_nnz", 1024)
    mats = [a1, a1, a2, a2, a3, a3]
    sizes = [p.n for p in plans]
    rng = np.random.default_rng(3)
    ids = rng.integers(0, len(plans), size=48)
    v64 = [vec_uniform(sizes[i], 900 + k) for k, i in enumerate(ids)]
    vs = [_vec(x, "f64") for x in v64]
    ref = []
    for i, v in zip(ids, vs):
        w = torch.empty_like(v)
        plans[i].apply(v, w)
        ref.append(w)
    torch.cuda.synchronize()
    srv = nap.Server(slots=3, max_batch=6)
    pids = [srv.add(p) for p in plans]
    outs = [torch.full_like(v, float("nan")) for v in vs]
    tickets = [srv.submit(pids[i], v, w) for i, v, w in zip(ids, vs, outs)]
    for t in tickets:
        srv.wait(t)
    torch.cuda.synchronize()
    for k, t in enumerate(tickets):
        _, _, bs = srv.info(t)
        if ids[k] in (2, 3):
            assert bs == 1                      # never batched
        assert torch.equal(outs[k], ref[k]), k
        i, a, p = int(ids[k]), mats[ids[k]], plans[ids[k]]
        got = outs[k].cpu().numpy()
        if i == 3:
            assert np.array_equal(got, oracle_spmv.spmv_split3(a, v64[k], p.n_p, p.ppn))
        elif i == 4:
            rows = p.rows()                     # position k holds row rows[k]
            v_nat = np.empty(a.n)
            v_nat[rows] = v64[k]
            w_nat = oracle_spmv.spmv_split(a, v_nat, p.n_p, strided=True)
            assert np.array_equal(got, w_nat[rows])
        else:
            assert np.array_equal(got, oracle_spmv.spmv_split(a, v64[k], p.n_p))
    srv.close()
    for p in plans:
        p.close()
