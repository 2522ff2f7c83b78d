"""The allocation-free apply (napspmv_apply_noalloc) through the C ABI.

Its workspace is the library's static per-GPU array, so two calls in a row
reuse memory that still holds the first call's ghosts and send buffer; the
second call here is on a smaller plan, so a stale value would show.  Each
result must equal, bit for bit, napspmv_apply_ws on the same plan and vector
with a fresh caller-owned workspace (same kernels), and the float64 ones the
oracle's split-order product.  A plan whose workspace exceeds the array is
refused with EUNSUPPORTED before anything runs.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_1612_08060_amd as nap
from oracle import spmv as oracle_spmv
from workloads import config, kkt_like, laplacian_2d, to_f32, vec_uniform

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _pair(so, a, v, n_p, ppn, mode, dtype):
    """(w from apply_noalloc, w from apply_ws with a fresh workspace)."""
    vals = a.val if dtype == "f64" else to_f32(a.val)
    p = nap.Plan(a.rowptr, a.col, vals, a.n, n_p, ppn, mode=mode, dtype=dtype)
    assert 0 < p.workspace_bytes <= so.napspmv_noalloc_max_workspace_bytes()
    tv = torch.from_numpy(v if dtype == "f64" else to_f32(v)).to(DEV)
    w_ref = torch.full_like(tv, float("nan"))
    w = torch.full_like(tv, float("nan"))
    ws = p.new_workspace()
    torch.cuda.synchronize()
    assert so.napspmv_apply_ws(p._h, _ptr(ws), _ptr(tv), _ptr(w_ref), _stream()) == 0, \
        so.napspmv_last_error()
    before = torch.cuda.memory_allocated()
    assert so.napspmv_apply_noalloc(p._h, _ptr(tv), _ptr(w), _stream()) == 0, \
        so.napspmv_last_error()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    p.close()
    return w.cpu().numpy().astype(np.float64), w_ref.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_equals_apply_ws_on_two_calls_second_smaller(dtype):
    so = nap.load_library()
    big = laplacian_2d(512, 512)                 # N = 262144, n_p 64 at ppn 4
    small = config(1)                            # 2D 64x64, n_p 16 at ppn 4
    v_big = vec_uniform(big.n, 21)
    for mode in ("nap", "standard"):
        for a, v, n_p, ppn in ((big, v_big, 64, 4), (small.csr, small.v, small.n_p, small.ppn)):
            w, w_ref = _pair(so, a, v, n_p, ppn, mode, dtype)
            assert np.array_equal(w, w_ref), (mode, a.n)
            if dtype == "f64":
                assert np.array_equal(w, oracle_spmv.spmv_split(a, v, n_p)), (mode, a.n)
            else:
                ref = oracle_spmv.spmv(a, v)
                assert np.linalg.norm(w - ref) / np.linalg.norm(ref) <= 1e-5, (mode, a.n)


def test_noalloc_refuses_a_plan_larger_than_its_workspace():
    so = nap.load_library()
    cap = so.napspmv_noalloc_max_workspace_bytes()
    assert cap == 64 << 20
    # uniformly random columns: nearly every entry is a ghost (about 12 M)
    a = kkt_like(1 << 21, 4, half_lo=3, half_hi=3, p_local=0.0)
    p = nap.Plan(a.rowptr, a.col, a.val, a.n, 512, 16)
    assert p.workspace_bytes > cap
    v = torch.zeros(a.n, dtype=torch.float64, device=DEV)
    w = torch.full_like(v, 7.0)
    rc = so.napspmv_apply_noalloc(p._h, _ptr(v), _ptr(w), _stream())
    assert rc == -4 and b"static workspace" in so.napspmv_last_error()
    torch.cuda.synchronize()
    assert bool(torch.all(w == 7.0))
    p.close()
