"""The byte counts behind bench.py's GB/s and roofline fields, on small
matrices: each term counted directly from the arrays it stands for, and the
two launches adding up to the whole apply plus the partial w round trip."""
import numpy as np
import pytest

import bench
import paper_1612_08060_amd as lib
from oracle import plan_ref
from workloads import config, random_pattern


@pytest.mark.parametrize("k,scale", [(1, 0), (2, 5), (3, 6)])
def test_byte_terms(k, scale):
    wl = config(k, scale=scale)
    a = wl.csr
    with lib.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, mode="standard",
                  row_starts=wl.row_starts, host_only=True) as p:
        st = p.stats
    n, nnz = a.n, a.nnz
    starts = np.asarray(wl.row_starts) if wl.row_starts is not None else None
    lay = plan_ref.Layout(n, wl.n_p, wl.ppn, starts)
    owner = np.array([lay.owner(j) for j in range(n)])
    rows = np.repeat(np.arange(n), np.diff(a.rowptr))
    off = owner[rows] != owner[a.col]
    ghosts = len({(int(t), int(j)) for t, j in zip(owner[rows][off], a.col[off])})
    assert st["ghosts"] == ghosts
    s_a = s_v = 8
    # values + int32 columns, two int32 row pointers, v, one read per ghost, w
    expect = nnz * (s_a + 4) + 2 * (n + 1) * 4 + n * s_v + ghosts * s_v + n * s_v
    assert bench.spmv_bytes(st, s_a, s_v) == expect
    # the standard gather: an index, a read of v and a write per ghost
    assert bench.exchange_bytes(st, s_v) == ghosts * (4 + 2 * s_v)
    r_off = int(np.unique(rows[off]).size)
    assert bench.rows_with_off_entries(a, wl.n_p, wl.row_starts) == r_off
    loc, rem = bench.launch_bytes(st, s_a, s_v, r_off)
    assert loc + rem == expect + ghosts * (4 + 2 * s_v) + 2 * r_off * s_v


def test_nap_exchange_terms():
    a = random_pattern(300, 0.03, seed=4)
    with lib.Plan(a.rowptr, a.col, a.val, a.n, 12, 4, mode="nap", host_only=True) as p:
        st = p.stats
    ph = st["phases"]
    e, g_on = ph["INTER"]["elems"], ph["L2"]["elems"]
    h = st["ghosts"] - g_on
    assert bench.exchange_bytes(st, 8) == e * 20 + h * 24 + g_on * 24
    assert bench.exchange_bytes(st, 8, exchange_copy=True) == e * 20 + h * 24 + g_on * 24 + 16 * e
    # direct reads: the pack alone (index, read of v, write per sent value)
    assert bench.exchange_bytes(st, 8, direct=True) == e * 20
    assert bench.exchange_bytes(st, 8, exchange_copy=True, direct=True) == e * 36
