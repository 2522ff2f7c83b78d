"""NAP plan variants (NAPSPMV_NAP_OWNER_MAP / SPLIT / DEDUP / THREE_WAY /
DIRECT) in the C-ABI host builder: every phase, every statistic and the
ghost lists equal the oracle's bit for bit, on random patterns,
paper-shaped matrices and the worked example.  Direct reads change only how
the device reads ghosts, so their messages are those of the same plan
without them."""
import numpy as np
import pytest

import paper_1612_08060_amd as lib
from oracle import plan_vec
from tests.helpers import example_2_1
from workloads import config, random_pattern

VARIANTS = [("owner_map",), ("split",), ("dedup",), ("owner_map", "split"),
            ("owner_map", "split", "dedup"), ("three_way",), ("split", "three_way"),
            ("direct",), ("dedup", "direct"), ("owner_map", "split", "dedup", "direct")]
FLAGS = {"owner_map": 0x4, "split": 0x8, "dedup": 0x10, "three_way": 0x20, "direct": 0x80}


def _compare(a, n_p, ppn, variant, row_starts=None):
    ref = plan_vec.plan(a, n_p, ppn, "nap", row_starts,
                        tuple(x for x in variant if x != "direct"))
    with lib.Plan(a.rowptr, a.col, a.val, a.n, n_p, ppn, mode="nap", row_starts=row_starts,
                  host_only=True, variant=variant) as p:
        assert p.variant == tuple(sorted(variant))
        st = p.stats
        assert st["flags"] == 0x1 | sum(FLAGS[v] for v in variant)
        for ph in lib.PHASES:
            got, exp = p.export(ph), ref["phases"][ph]
            for g, e in zip(got, exp):
                assert np.array_equal(g, e), (ph, variant)
            assert st["phases"][ph] == plan_vec.phase_stats(exp, n_p), ph
        gp, gc = p.ghosts()
        assert np.array_equal(gc, ref["ghost_j"])
    return st


@pytest.mark.parametrize("variant", VARIANTS)
def test_example_2_1(variant):
    g, a = example_2_1()
    _compare(a, 6, 2, variant)


@pytest.mark.parametrize("n_p,ppn", [(2, 2), (4, 2), (6, 3), (8, 4), (8, 2), (12, 4), (9, 3),
                                     (16, 8), (16, 4), (24, 8)])
@pytest.mark.parametrize("variant", VARIANTS)
def test_random_patterns(n_p, ppn, variant):
    for seed in range(3):
        a = random_pattern(30 + 9 * n_p + 7 * seed, 0.03 + 0.05 * seed,
                           seed=500 + 31 * n_p + ppn + seed, empty_rows=seed, duplicates=seed)
        _compare(a, n_p, ppn, variant)


@pytest.mark.parametrize("variant", VARIANTS)
def test_explicit_row_starts(variant):
    a = random_pattern(120, 0.05, seed=77)
    starts = np.array([0, 3, 20, 21, 40, 64, 90, 100, 120], np.int64)
    _compare(a, 8, 4, variant, starts)


@pytest.mark.parametrize("k,scale", [(1, 0), (2, 4), (3, 4), (4, 2)])
@pytest.mark.parametrize("variant", VARIANTS)
def test_paper_shaped_configs(k, scale, variant):
    wl = config(k, scale=scale)
    _compare(wl.csr, wl.n_p, wl.ppn, variant, wl.row_starts)


def test_variants_keep_inter_node_volume():
    """E(n, m) does not depend on the variant: the inter-node element count
    is the same, and the default plan's L1 volume too unless split moves
    receivers."""
    wl = config(2, scale=4)
    base = _compare(wl.csr, wl.n_p, wl.ppn, ())
    for variant in VARIANTS:
        st = _compare(wl.csr, wl.n_p, wl.ppn, variant)
        assert st["phases"]["INTER"]["elems"] == base["phases"]["INTER"]["elems"]
        if "split" not in variant:
            assert st["phases"]["L1"] == base["phases"]["L1"]
        assert (st["nnz_on"], st["nnz_off"], st["ghosts"]) == (
            base["nnz_on"], base["nnz_off"], base["ghosts"])


def test_variant_flags_rejected_for_standard_and_unknown():
    a = random_pattern(20, 0.2, seed=3)
    with pytest.raises(lib.NapspmvError) as e:
        lib.Plan(a.rowptr, a.col, a.val, a.n, 4, 2, mode="standard", host_only=True,
                 variant=("split",))
    assert e.value.code == -1
    with pytest.raises(ValueError):
        lib.Plan(a.rowptr, a.col, a.val, a.n, 4, 2, mode="nap", host_only=True,
                 variant=("nope",))


def test_direct_rejected_with_three_way_and_standard():
    a = random_pattern(20, 0.2, seed=4)
    for mode, variant in (("nap", ("direct", "three_way")), ("standard", ("direct",))):
        with pytest.raises(lib.NapspmvError) as e:
            lib.Plan(a.rowptr, a.col, a.val, a.n, 4, 2, mode=mode, host_only=True,
                     variant=variant)
        assert e.value.code == -1
