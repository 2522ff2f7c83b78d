"""Third hierarchy level (on-socket / off-socket message statistics): the
library's split of every phase equals the oracle's, and the split behaves as
its definition requires at the extremes."""
import numpy as np
import pytest

import paper_1612_08060_amd as lib
from oracle import plan_vec
from workloads import config, random_pattern


def _check(a, n_p, ppn, mode, pps, strided=False, row_starts=None):
    ref = plan_vec.plan(a, n_p, ppn, mode, row_starts, strided=strided)
    with lib.Plan(a.rowptr, a.col, a.val, a.n, n_p, ppn, mode=mode, host_only=True,
                  strided=strided, row_starts=row_starts) as p:
        got = p.level_stats(pps)
        total = p.stats["phases"]
    for ph in lib.PHASES:
        exp = plan_vec.level_stats(ref["phases"][ph], n_p, pps)
        assert got[ph] == exp, ph
        for k in ("msgs", "elems"):
            assert got[ph]["on_socket"][k] + got[ph]["off_socket"][k] == total[ph][k]
    return got


@pytest.mark.parametrize("n_p,ppn,pps", [(8, 4, 2), (12, 4, 1), (12, 4, 4), (16, 8, 2), (16, 8, 4)])
@pytest.mark.parametrize("mode", ["standard", "nap"])
def test_random_patterns(n_p, ppn, pps, mode):
    for seed in range(3):
        a = random_pattern(40 + 9 * n_p + seed, 0.05 + 0.03 * seed, seed=n_p * 13 + seed)
        _check(a, n_p, ppn, mode, pps)


@pytest.mark.parametrize("mode", ["standard", "nap"])
def test_extremes(mode):
    wl = config(2, scale=4)
    a = wl.csr
    whole = _check(a, wl.n_p, wl.ppn, mode, wl.ppn)       # one socket per node
    for ph in ("L0", "L1", "L2"):
        assert whole[ph]["off_socket"]["msgs"] == 0
    single = _check(a, wl.n_p, wl.ppn, mode, 1)           # one process per socket
    for ph in lib.PHASES:
        assert single[ph]["on_socket"]["msgs"] == 0
    assert whole["INTER"]["on_socket"]["msgs"] == 0       # inter-node is never on-socket


def test_paper_shapes_and_strided():
    wl = config(3, scale=5)
    _check(wl.csr, wl.n_p, wl.ppn, "nap", 8)
    _check(wl.csr, wl.n_p, wl.ppn, "nap", 8, strided=True)
    wl = config(4, scale=3)
    _check(wl.csr, wl.n_p, wl.ppn, "standard", 4, row_starts=wl.row_starts)


def test_bad_socket_size():
    a = random_pattern(30, 0.1, seed=1)
    with lib.Plan(a.rowptr, a.col, a.val, a.n, 6, 3, mode="nap", host_only=True) as p:
        for bad in (0, 2, 4):
            with pytest.raises(lib.NapspmvError):
                p.level_stats(bad)
