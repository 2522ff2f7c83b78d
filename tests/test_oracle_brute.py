"""The literal oracle against brute force on tiny random matrices, and the
vectorised oracle against the literal one.

Brute force evaluates each definition from its quantifiers over a dense
pattern (P, D of section 2.1; N, E, I and the three J sets of section 4).
Matrices are non-symmetric, include empty rows, duplicate entries and stored
zeros, and every ppn dividing n_p is tried, including the uneven remainder
block and explicit block boundaries.
"""
import itertools

import numpy as np
import pytest

from oracle import brute, plan_ref, plan_vec, simulate
from tests.helpers import arrays_to_triples, triples
from workloads import CSR, random_pattern

CASES = []
for n_p in range(1, 9):
    for ppn in [d for d in range(1, n_p + 1) if n_p % d == 0]:
        CASES.append((n_p, ppn))


def _matrix(n, seed, zeros=False):
    a = random_pattern(n, density=0.12 + 0.02 * (seed % 5), seed=seed,
                       empty_rows=seed % 3, duplicates=seed % 4)
    if zeros:
        a = CSR(a.n, a.rowptr, a.col, np.where(np.arange(a.nnz) % 5 == 0, 0.0, a.val))
    return a


@pytest.mark.parametrize("n_p,ppn", CASES)
def test_literal_vs_brute(n_p, ppn):
    for seed in range(3):
        n = 9 + 7 * seed + n_p          # N not a multiple of n_p in most cases
        a = _matrix(n, 100 * n_p + 10 * ppn + seed, zeros=seed == 1)
        lay = plan_ref.Layout(n, n_p, ppn)
        s = plan_ref.standard_plan(a, lay)
        b = brute.standard_sets(a, n_p, ppn)
        assert s["P"] == b["P"]
        assert s["D"] == b["D"]
        nap = plan_ref.nap_plan(a, lay)
        bn = brute.nap_sets(a, n_p, ppn)
        assert nap["N"] == bn["N"] and nap["E"] == bn["E"]
        assert nap["t_rank"] == bn["send_rank"] and nap["u_rank"] == bn["recv_rank"]
        assert triples(nap["phases"]["INTER"]) == triples(
            (x, y, v) for (x, y), v in bn["I"].items())
        for key, ph in (("J0", "L0"), ("J1", "L1"), ("J2", "L2")):
            assert triples(nap["phases"][ph]) == triples(
                (x, y, v) for (x, y), v in bn[key].items()), (key, n_p, ppn, seed)


@pytest.mark.parametrize("n_p,ppn", CASES)
def test_vectorised_vs_literal(n_p, ppn):
    for seed in range(3):
        n = 11 + 13 * seed + 2 * n_p
        a = _matrix(n, 7 + 1000 * n_p + 10 * ppn + seed)
        lay = plan_ref.Layout(n, n_p, ppn)
        for mode in ("standard", "nap"):
            lit = plan_ref.plan(a, lay, mode)
            vec = plan_vec.plan(a, n_p, ppn, mode)
            for ph in plan_ref.PHASES:
                assert arrays_to_triples(vec["phases"][ph]) == triples(lit["phases"][ph])


def test_explicit_row_starts():
    a = _matrix(40, 5)
    starts = [0, 3, 4, 11, 20, 21, 33, 38, 40]
    lay = plan_ref.Layout(40, 8, 4, row_starts=starts)
    b = brute.nap_sets(a, 8, 4, row_starts=starts)
    nap = plan_ref.nap_plan(a, lay)
    assert nap["E"] == b["E"]
    for key, ph in (("J0", "L0"), ("J1", "L1"), ("J2", "L2")):
        assert triples(nap["phases"][ph]) == triples((x, y, v) for (x, y), v in b[key].items())
    for mode in ("standard", "nap"):
        vec = plan_vec.plan(a, 8, 4, mode, given_starts=starts)
        lit = plan_ref.plan(a, lay, mode)
        for ph in plan_ref.PHASES:
            assert arrays_to_triples(vec["phases"][ph]) == triples(lit["phases"][ph])


@pytest.mark.parametrize("n_p,ppn", [(4, 2), (6, 3), (8, 2), (8, 4), (6, 1), (6, 6)])
def test_every_ghost_delivered_once(n_p, ppn):
    for seed in range(4):
        n = 20 + 5 * seed
        a = _matrix(n, 31 * seed + n_p * ppn)
        lay = plan_ref.Layout(n, n_p, ppn)
        v = np.random.default_rng(seed).standard_normal(n)
        _, w_s = simulate.simulate_standard(a, lay, plan_ref.standard_plan(a, lay), v)
        _, w_n = simulate.simulate_nap(a, lay, plan_ref.nap_plan(a, lay), v)
        ref = brute.matvec(a, v)
        assert np.allclose(w_s, ref, rtol=1e-13, atol=1e-13)
        assert np.allclose(w_n, ref, rtol=1e-13, atol=1e-13)
        # the simulation's per-rank products, from delivered values, equal the
        # C split-order routines bit for bit (two independent evaluations)
        from oracle import spmv as ospmv
        assert np.array_equal(w_s, ospmv.spmv_split(a, v, n_p))
        assert np.array_equal(w_n, ospmv.spmv_split(a, v, n_p))
        _, w_3 = simulate.simulate_nap(a, lay, plan_ref.nap_plan(a, lay, ("three_way",)), v)
        assert np.array_equal(w_3, ospmv.spmv_split3(a, v, n_p, ppn))


def test_mapping_invariants_many_partners():
    """More partner nodes than processes per node (the paper is silent):
    each partner is assigned exactly once, and per-process partner counts
    differ by at most one, both for sending (T) and receiving (U)."""
    a = random_pattern(96, 0.08, seed=3)
    n_p, ppn = 24, 2                      # 12 nodes, up to 11 partners each
    lay = plan_ref.Layout(96, n_p, ppn)
    nap = plan_ref.nap_plan(a, lay)
    for n in range(lay.n_nodes):
        ranks = [lay.rank(p, n) for p in range(ppn)]
        sent = list(itertools.chain.from_iterable(nap["T"][r] for r in ranks))
        assert sorted(sent) == nap["N"][n]
        cnt = [len(nap["T"][r]) for r in ranks]
        assert max(cnt) - min(cnt) <= 1
        senders = [m for m in range(lay.n_nodes) if n in nap["N"][m]]
        got = list(itertools.chain.from_iterable(nap["U"][r] for r in ranks))
        assert sorted(got) == senders
        cnt = [len(nap["U"][r]) for r in ranks]
        assert max(cnt) - min(cnt) <= 1


@pytest.mark.parametrize("n_p,ppn", [(2, 1), (4, 2), (6, 3), (8, 4), (6, 2)])
def test_strided_literal_vs_brute_and_vectorised(n_p, ppn):
    """Strided partition (row r on process r mod n_p): the literal sets equal
    the brute-force quantifiers and the vectorised evaluation, and every
    ghost is delivered once with the owner's value."""
    from oracle import brute, plan_ref, plan_vec, simulate
    from tests.helpers import arrays_to_triples, triples
    for seed in range(3):
        n = 19 + 5 * n_p + seed
        a = random_pattern(n, 0.15, seed=70 + 7 * n_p + seed, empty_rows=1, duplicates=2)
        lay = plan_ref.Layout(n, n_p, ppn, strided=True)
        std = plan_ref.standard_plan(a, lay)
        b = brute.standard_sets(a, n_p, ppn, strided=True)
        assert std["P"] == b["P"] and std["D"] == {k: v for k, v in b["D"].items()}
        nap = plan_ref.nap_plan(a, lay)
        bn = brute.nap_sets(a, n_p, ppn, strided=True)
        assert triples(nap["phases"]["INTER"]) == triples([(s, q, idx) for (s, q), idx in bn["I"].items()])
        for ph, J in (("L0", "J0"), ("L1", "J1"), ("L2", "J2")):
            assert triples(nap["phases"][ph]) == triples([(p, s, idx) for (p, s), idx in bn[J].items()])
        for mode, lit in (("standard", std), ("nap", nap)):
            vec = plan_vec.plan(a, n_p, ppn, mode, strided=True)
            for ph in plan_ref.PHASES:
                assert arrays_to_triples(vec["phases"][ph]) == triples(lit["phases"][ph]), (mode, ph)
        v = np.random.default_rng(seed).standard_normal(n)
        simulate.simulate_standard(a, lay, std, v)
        simulate.simulate_nap(a, lay, nap, v)


def test_strided_is_a_symmetric_permutation_of_contiguous():
    """Renumbering row r to its position in process-major order (process
    r mod n_p, slot r div n_p) turns the strided plan into the contiguous plan
    of the permuted matrix, message for message."""
    from oracle import plan_ref
    from tests.helpers import csr_from_rows, triples
    n, n_p, ppn = 37, 6, 2
    a = random_pattern(n, 0.12, seed=5, duplicates=1)
    counts = [len(range(p, n, n_p)) for p in range(n_p)]
    starts = np.concatenate([[0], np.cumsum(counts)])
    new = np.array([starts[r % n_p] + r // n_p for r in range(n)])
    old_of = np.argsort(new)
    rows = [[int(new[c]) for c in a.col[a.rowptr[o]:a.rowptr[o + 1]]] for o in old_of]
    b = csr_from_rows(rows)
    lay_s = plan_ref.Layout(n, n_p, ppn, strided=True)
    lay_c = plan_ref.Layout(n, n_p, ppn, row_starts=starts)
    for mode in ("standard", "nap"):
        ps = plan_ref.plan(a, lay_s, mode)
        pc = plan_ref.plan(b, lay_c, mode)
        for ph in plan_ref.PHASES:
            mapped = [(s, d, tuple(sorted(int(new[j]) for j in idx))) for s, d, idx in ps["phases"][ph]]
            assert triples(mapped) == triples(pc["phases"][ph]), (mode, ph)
