"""Strided partition (NAPSPMV_PARTITION_STRIDED, row r on process r mod n_p)
in the host builder: after renumbering the oracle's sets (computed directly
with the strided owner map) into process-major order, every phase, every
statistic and every ghost list equals the library's."""
import numpy as np
import pytest

import paper_1612_08060_amd as lib
from oracle import plan_vec
from workloads import config, random_pattern


def _expected_positions(n, n_p):
    counts = np.array([len(range(p, n, n_p)) for p in range(n_p)])
    starts = np.concatenate([[0], np.cumsum(counts)])
    r = np.arange(n)
    return starts[r % n_p] + r // n_p


def _compare(a, n_p, ppn, mode, variant=()):
    ref = plan_vec.plan(a, n_p, ppn, mode, None, variant, strided=True)
    with lib.Plan(a.rowptr, a.col, a.val, a.n, n_p, ppn, mode=mode, host_only=True,
                  variant=variant, strided=True) as p:
        rows = p.rows()
        new = np.empty(a.n, np.int64)
        new[rows] = np.arange(a.n)
        assert np.array_equal(new, _expected_positions(a.n, n_p))
        st = p.stats
        for ph in lib.PHASES:
            src, dst, ptr, idx = ref["phases"][ph]
            g = p.export(ph)
            assert np.array_equal(g[0], src) and np.array_equal(g[1], dst)
            assert np.array_equal(g[2], ptr)
            for k in range(len(src)):
                assert np.array_equal(g[3][ptr[k]:ptr[k + 1]], np.sort(new[idx[ptr[k]:ptr[k + 1]]]))
            assert st["phases"][ph] == plan_vec.phase_stats(ref["phases"][ph], n_p), ph
        gp, gc = p.ghosts()
        t, j = ref["ghost_t"], ref["ghost_j"]
        assert np.array_equal(np.diff(gp), np.bincount(t, minlength=n_p))
        for r in range(n_p):
            assert np.array_equal(gc[gp[r]:gp[r + 1]], np.sort(new[j[t == r]]))
        rows_i = np.repeat(np.arange(a.n), np.diff(a.rowptr))
        on = (rows_i % n_p) == (a.col % n_p)
        assert st["nnz_on"] == int(on.sum()) and st["nnz_off"] == int((~on).sum())
    return st


@pytest.mark.parametrize("n_p,ppn", [(1, 1), (2, 1), (4, 2), (6, 3), (8, 4), (12, 4), (16, 8)])
@pytest.mark.parametrize("mode", ["standard", "nap"])
def test_random_patterns(n_p, ppn, mode):
    for seed in range(3):
        a = random_pattern(20 + 11 * n_p + seed, 0.04 + 0.04 * seed, seed=41 * n_p + seed,
                           empty_rows=seed, duplicates=seed)
        _compare(a, n_p, ppn, mode)


@pytest.mark.parametrize("variant", [("owner_map",), ("dedup",), ("three_way",),
                                     ("owner_map", "dedup", "three_way")])
def test_variants(variant):
    for seed in range(2):
        a = random_pattern(150 + seed, 0.05, seed=seed + 8, duplicates=2)
        _compare(a, 12, 4, "nap", variant)


@pytest.mark.parametrize("k,scale", [(1, 0), (2, 4), (3, 5), (4, 3)])
@pytest.mark.parametrize("mode", ["standard", "nap"])
def test_paper_shaped_matrices(k, scale, mode):
    wl = config(k, scale=scale)
    _compare(wl.csr, wl.n_p, wl.ppn, mode)


def test_strided_spreads_ghosts():
    """On the KKT-like matrix the strided partition multiplies the ghosts,
    and NAP's node aggregation removes most inter-node messages."""
    wl = config(3, scale=5)
    a = wl.csr
    with lib.Plan(a.rowptr, a.col, a.val, a.n, wl.n_p, wl.ppn, "standard", host_only=True) as p:
        cont = p.stats
    s_std = _compare(a, wl.n_p, wl.ppn, "standard")
    s_nap = _compare(a, wl.n_p, wl.ppn, "nap")
    assert s_std["ghosts"] > 2 * cont["ghosts"]
    assert s_nap["phases"]["INTER"]["msgs"] * 4 < s_std["phases"]["INTER"]["msgs"]


def test_rows_identity_and_errors():
    a = random_pattern(30, 0.1, seed=2)
    with lib.Plan(a.rowptr, a.col, a.val, a.n, 3, 1, host_only=True) as p:
        assert np.array_equal(p.rows(), np.arange(30))
    with pytest.raises(lib.NapspmvError) as e:
        lib.Plan(a.rowptr, a.col, a.val, a.n, 3, 1, host_only=True, strided=True,
                 row_starts=np.array([0, 10, 20, 30], np.int64))
    assert e.value.code == -1
    with pytest.raises(lib.NapspmvError) as e:
        lib.Plan(a.rowptr, a.col, a.val, a.n, 4, 2, mode="nap", host_only=True, strided=True,
                 variant=("split",))
    assert e.value.code == -1
