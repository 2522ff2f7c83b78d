"""Plans with a third hierarchy level (napspmv_plan_create_sockets) built on
the host: every phase, the four parts of each intra-node step's socket
route, and every statistic equal the oracle's bit for bit (plan_vec, itself
pinned against the literal and brute-force evaluations), including uneven
blocks, remainder rows and the strided partition; argument checks."""
import ctypes

import numpy as np
import pytest

import paper_1612_08060_amd as lib
from oracle import plan_vec
from tests.helpers import arrays_to_triples
from workloads import config, random_pattern


def _check(a, n_p, ppn, pps, row_starts=None, strided=False):
    """The library's phases equal the oracle's; a strided plan's indices are
    in process-major order, so the oracle's are renamed first (the sets only
    depend on which process owns which index)."""
    ref = plan_vec.socket_plan(a, n_p, ppn, pps, row_starts, strided=strided)
    with lib.Plan(a.rowptr, a.col, a.val, a.n, n_p, ppn, mode="nap", host_only=True,
                  sockets=pps, row_starts=row_starts, strided=strided) as p:
        new = np.empty(a.n, np.int64)
        new[p.rows()] = np.arange(a.n)
        for ph in lib.PHASES + lib.SOCKET_PHASES:
            want = [(s, d, tuple(sorted(int(new[j]) for j in idx)))
                    for s, d, idx in arrays_to_triples(ref["phases"][ph])]
            assert arrays_to_triples(p.export(ph)) == want, ph
        ss = p.socket_stats()
        for ph in lib.SOCKET_PHASES:
            assert ss[ph] == plan_vec.phase_stats(ref["phases"][ph], n_p), ph
        st = p.stats["phases"]
        for ph in lib.PHASES:
            assert st[ph] == plan_vec.phase_stats(ref["phases"][ph], n_p), ph


@pytest.mark.parametrize("n_p,ppn,pps", [(8, 4, 2), (12, 6, 2), (12, 6, 3), (16, 8, 2), (16, 8, 4),
                                         (16, 4, 1), (16, 4, 4)])
def test_random_patterns(n_p, ppn, pps):
    for seed in range(3):
        a = random_pattern(50 + 9 * n_p + seed, 0.04 + 0.03 * seed, seed=n_p * 17 + seed,
                           empty_rows=2, duplicates=3)
        _check(a, n_p, ppn, pps)


def test_uneven_blocks_remainder_and_strided():
    a = random_pattern(203, 0.05, seed=5)
    _check(a, 16, 8, 4)                                   # 203 = 16 * 12 + 11
    wl = config(4, scale=3)
    _check(wl.csr, wl.n_p, wl.ppn, 4, row_starts=wl.row_starts)
    _check(random_pattern(150, 0.05, seed=8), 12, 6, 3, strided=True)


def test_paper_shapes():
    wl = config(2, scale=3)
    _check(wl.csr, wl.n_p, wl.ppn, 8)
    wl = config(3, scale=6)
    _check(wl.csr, wl.n_p, wl.ppn, 8)
    _check(wl.csr, wl.n_p, wl.ppn, 4)


def test_argument_checks():
    so = lib.load_library()
    a = random_pattern(40, 0.1, seed=1)
    rp, col, val = a.rowptr, a.col, a.val
    h = ctypes.c_void_p()

    def make(pps, flags=0x1, n_p=8, ppn=4):
        return so.napspmv_plan_create_sockets(rp.ctypes.data, col.ctypes.data, val.ctypes.data,
                                              0, a.n, n_p, ppn, pps, None, flags,
                                              ctypes.byref(h), None)
    assert make(0) == -1 and not h.value
    assert make(3) == -1 and b"divide" in so.napspmv_last_error()
    assert make(2, flags=0x1 | 0x4) == -1               # a NAP variant
    assert make(2, flags=0x1 | 0x2) == -1               # the explicit hop
    assert make(2) == 0 and h.value
    pps = ctypes.c_int64()
    assert so.napspmv_plan_socket_stats(h, ctypes.byref(pps), None) == 0 and pps.value == 2
    so.napspmv_plan_destroy(h)
    with lib.Plan(rp, col, val, a.n, 8, 4, mode="nap", host_only=True) as p:
        with pytest.raises(lib.NapspmvError):
            p.socket_stats()
        with pytest.raises(lib.NapspmvError):
            p.export("L2_cross")
        assert so.napspmv_plan_socket_stats(p._h, ctypes.byref(pps), None) == 0 and pps.value == 0
    with pytest.raises(ValueError):
        lib.Plan(rp, col, val, a.n, 8, 4, mode="standard", host_only=True, sockets=2)
