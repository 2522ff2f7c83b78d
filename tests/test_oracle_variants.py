"""Pins of the NAPSpMV plan variants (section 4.1: the owner mapping and the
split of a partner over several processes; cross-step deduplication of the
fully local step).

Hand-derived values on Example 2.1, brute-force minimality of the owner
mapping, the piece structure of the split, and, for every variant, delivery of
every ghost exactly once with the owner's value.
"""
import itertools

import numpy as np
import pytest

from oracle import plan_ref as R
from oracle import plan_vec as V
from oracle import simulate as S
from tests.helpers import arrays_to_triples, example_2_1, triples
from workloads import random_pattern

VARIANTS = [(), ("owner_map",), ("dedup",), ("split",), ("split", "owner_map"),
            ("owner_map", "dedup", "split")]


@pytest.fixture(scope="module")
def ex():
    g, a = example_2_1()
    return R.Layout(6, 6, 2), a


def test_example_owner_map(ex):
    # E(0,1) = {0, 1}: ranks 0 and 1 hold one index each -> the lower, rank 0.
    # E(0,2) = {0}: rank 0.  E(1,0) = {3}: rank 3.  E(1,2) = {2}: rank 2.
    # E(2,0) = {4, 5}: tie -> rank 4.  Receivers follow the printed U table:
    # (0,1) -> 3, (0,2) -> 5, (1,0) -> 1, (1,2) -> 4, (2,0) -> 0.
    lay, a = ex
    p = R.nap_plan(a, lay, ("owner_map",))
    assert triples(p["phases"]["INTER"]) == [
        (0, 3, (0, 1)), (0, 5, (0,)), (2, 4, (2,)), (3, 1, (3,)), (4, 0, (4, 5))]
    # Only v_1 (sent by rank 0 for node 1) and v_5 (sent by rank 4) are not
    # owned by their sender.
    assert triples(p["phases"]["L0"]) == [(1, 0, (1,)), (5, 4, (5,))]
    base = R.nap_plan(a, lay)
    for ph in ("L1", "L2"):
        assert triples(p["phases"][ph]) == triples(base["phases"][ph])


def test_example_split(ex):
    # Node 2 has one partner (node 0) and two processes: E(2,0) = {4, 5} is
    # cut into {4} sent by rank 4 and {5} sent by rank 5.  Node 0 has two
    # senders, so rank 0 alone receives both pieces.  Nodes 0 and 1 have two
    # partners each and keep the default mapping (T printed in the paper).
    lay, a = ex
    p = R.nap_plan(a, lay, ("split",))
    assert triples(p["phases"]["INTER"]) == [
        (0, 3, (0, 1)), (1, 5, (0,)), (2, 1, (3,)), (3, 4, (2,)), (4, 0, (4,)), (5, 0, (5,))]
    # The default plan's (5, 4, {5}) hand-over disappears: rank 5 sends its own.
    assert triples(p["phases"]["L0"]) == [
        (0, 1, (0,)), (1, 0, (1,)), (2, 3, (2,)), (3, 2, (3,))]


def test_example_dedup(ex):
    # On-node ghosts: rank 0 needs v_1, rank 2 needs v_3, rank 3 needs v_2.
    # Each of them already travels between the same two ranks in the
    # on_node -> off_node step, so the fully local step is empty.
    lay, a = ex
    p = R.nap_plan(a, lay, ("dedup",))
    base = R.nap_plan(a, lay)
    assert triples(base["phases"]["L2"]) == [(1, 0, (1,)), (2, 3, (2,)), (3, 2, (3,))]
    assert p["phases"]["L2"] == []
    for ph in ("INTER", "L0", "L1"):
        assert triples(p["phases"][ph]) == triples(base["phases"][ph])


def _cases():
    out = []
    for n_p, ppn in [(4, 2), (6, 3), (8, 4), (8, 2), (12, 4), (9, 3), (16, 8)]:
        for seed in range(2):
            n = 24 + 7 * n_p + 5 * seed
            out.append((n_p, ppn, seed, n))
    return out


def _matrix(n_p, ppn, seed, n):
    return random_pattern(n, 0.05 + 0.04 * seed, 11 + 97 * n_p + 13 * ppn + seed,
                          empty_rows=seed, duplicates=1)


@pytest.mark.parametrize("n_p,ppn,seed,n", _cases())
@pytest.mark.parametrize("variant", VARIANTS)
def test_vectorised_equals_literal(n_p, ppn, seed, n, variant):
    a = _matrix(n_p, ppn, seed, n)
    lit = R.nap_plan(a, R.Layout(n, n_p, ppn), variant)
    vec = V.nap_plan(a, n_p, ppn, None, variant)
    for ph in R.PHASES:
        assert arrays_to_triples(vec["phases"][ph]) == triples(lit["phases"][ph]), ph


@pytest.mark.parametrize("n_p,ppn,seed,n", _cases())
@pytest.mark.parametrize("variant", VARIANTS)
def test_delivery(n_p, ppn, seed, n, variant):
    a = _matrix(n_p, ppn, seed, n)
    lay = R.Layout(n, n_p, ppn)
    v = np.random.default_rng(seed).standard_normal(n)
    _, w = S.simulate_nap(a, lay, R.nap_plan(a, lay, variant), v)
    _, w0 = S.simulate_nap(a, lay, R.nap_plan(a, lay), v)
    assert w.tobytes() == w0.tobytes()


@pytest.mark.parametrize("n_p,ppn,seed,n", _cases())
def test_owner_map_sender_holds_most(n_p, ppn, seed, n):
    """Brute force over every local process of n: the chosen sender owns the
    most indices of E(n, m), the lowest local number on ties."""
    a = _matrix(n_p, ppn, seed, n)
    lay = R.Layout(n, n_p, ppn)
    N, E = R.node_sets(a, lay)
    p = R.nap_plan(a, lay, ("owner_map",))
    sender = {}
    for s, q, idx in p["phases"]["INTER"]:
        sender[(lay.node(s), lay.node(q))] = s
    assert set(sender) == set(E)
    for (nd, m), idx in E.items():
        held = [sum(lay.owner(j) == lay.rank(x, nd) for j in idx) for x in range(ppn)]
        best = max(held)
        assert sender[(nd, m)] == lay.rank(min(x for x in range(ppn) if held[x] == best), nd)


@pytest.mark.parametrize("n_p,ppn,seed,n", _cases())
def test_split_pieces(n_p, ppn, seed, n):
    """Pieces of E(n, m) are disjoint, cover it, are contiguous in index order
    with lengths differing by at most one, and a node with k < ppn partners
    spreads them over ceil((ppn - i) / k) senders."""
    a = _matrix(n_p, ppn, seed, n)
    lay = R.Layout(n, n_p, ppn)
    N, E = R.node_sets(a, lay)
    p = R.nap_plan(a, lay, ("split",))
    pieces = {}
    for s, q, idx in p["phases"]["INTER"]:
        pieces.setdefault((lay.node(s), lay.node(q)), []).append((s, q, list(idx)))
    assert set(pieces) == set(E)
    for (nd, m), ps in pieces.items():
        ps.sort(key=lambda x: x[2][0])
        flat = [j for _, _, idx in ps for j in idx]
        assert flat == sorted(E[(nd, m)])
        lens = [len(idx) for _, _, idx in ps]
        assert max(lens) - min(lens) <= 1
        k = len(N[nd])
        if k >= ppn:
            assert len(ps) == 1
        else:
            order = sorted(N[nd], key=lambda x: (-len(E[(nd, x)]), x))
            i = order.index(m)
            n_snd = len(range(i, ppn, k))
            assert len(ps) == min(n_snd, len(E[(nd, m)]))
            assert [lay.local(s) for s, _, _ in ps] == list(range(i, ppn, k))[:len(ps)]


def test_split_every_process_sends():
    """A node with fewer partners than processes, each partner needing at
    least ppn values, has every one of its processes send off-node."""
    n_p, ppn = 8, 4            # two nodes: each node's only partner is the other
    n = 64
    rng = np.random.default_rng(3)
    rows = []
    for i in range(n):
        other = (np.arange(32) + 32 * (1 - i // 32))
        rows.append(sorted({i} | set(rng.choice(other, 6, replace=False).tolist())))
    from tests.helpers import csr_from_rows
    a = csr_from_rows(rows)
    lay = R.Layout(n, n_p, ppn)
    N, E = R.node_sets(a, lay)
    assert all(len(E[k]) >= ppn for k in E) and all(len(N[x]) == 1 for x in range(2))
    base = R.nap_plan(a, lay)
    p = R.nap_plan(a, lay, ("split",))
    senders = {s for s, _, _ in p["phases"]["INTER"]}
    receivers = {q for _, q, _ in p["phases"]["INTER"]}
    assert senders == set(range(n_p)) and receivers == set(range(n_p))
    assert len({s for s, _, _ in base["phases"]["INTER"]}) == 2


@pytest.mark.parametrize("n_p,ppn,seed,n", _cases())
def test_dedup_covers_and_is_disjoint(n_p, ppn, seed, n):
    """Under dedup the fully local step and the on_node -> off_node step share
    no (src, dst, j), and together carry every on-node ghost D(r, t)."""
    a = _matrix(n_p, ppn, seed, n)
    lay = R.Layout(n, n_p, ppn)
    p = R.nap_plan(a, lay, ("dedup",))
    l2 = {(s, d, j) for s, d, idx in p["phases"]["L2"] for j in idx}
    l0 = {(s, d, j) for s, d, idx in p["phases"]["L0"] for j in idx}
    assert not (l2 & l0)
    std = R.plan(a, lay, "standard")
    need = {(s, d, j) for s, d, idx in std["phases"]["L2"] for j in idx}
    assert need <= (l2 | l0)
    assert l2 <= need


@pytest.mark.parametrize("variant", VARIANTS[1:])
def test_simulation_catches_a_dropped_piece(ex, variant):
    """A plan with one INTER index removed fails delivery, under every variant."""
    lay, a = ex
    p = R.nap_plan(a, lay, variant)
    s, q, idx = p["phases"]["INTER"][0]
    broken = dict(p)
    broken["phases"] = dict(p["phases"])
    broken["phases"]["INTER"] = [(s, q, tuple(idx)[1:])] + list(p["phases"]["INTER"][1:])
    with pytest.raises(S.DeliveryError):
        S.simulate_nap(a, lay, broken, np.arange(6, dtype=np.float64) + 0.5)


def test_unknown_variant_rejected(ex):
    lay, a = ex
    with pytest.raises(ValueError):
        R.nap_plan(a, lay, ("nope",))
    with pytest.raises(ValueError):
        V.nap_plan(a, 6, 2, None, ("nope",))
