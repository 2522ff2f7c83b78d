"""The oracle against the worked example of section 2 (Example 2.1) and every
table the paper prints for it (sections 2.1, 4.1, 4.2).

Printed tables that agree with the definitions are exact pins.  Four tables
(I and the three local steps) disagree with the definitions; the golden file
records the printed and the corrected sets with the reason for each
correction, and the tests check both that the oracle gives the corrected sets
and that the correction touches only the entries named there.
"""
import numpy as np
import pytest

from oracle import brute, plan_ref, plan_vec, simulate, spmv
from workloads import CSR
from tests.helpers import arrays_to_triples, example_2_1, triples


@pytest.fixture(scope="module")
def ex():
    g, a = example_2_1()
    lay = plan_ref.Layout(g["layout"]["N"], g["layout"]["n_p"], g["layout"]["ppn"])
    return g, a, lay


def _as_int_dict(d):
    return {int(k): list(v) for k, v in d.items()}


def test_rank_tuples(ex):
    _, _, lay = ex
    # rank r = (r mod ppn, r div ppn)  (section 2, SMP-style ordering)
    assert [(lay.local(r), lay.node(r)) for r in range(6)] == [
        (0, 0), (1, 0), (0, 1), (1, 1), (0, 2), (1, 2)]


def test_standard_sets_match_printed_tables(ex):
    g, a, lay = ex
    s = plan_ref.standard_plan(a, lay)
    assert s["P"] == _as_int_dict(g["printed"]["P"]["value"])
    assert triples((r, t, v) for (r, t), v in s["D"].items()) == triples(
        g["printed"]["D"]["value"])


def test_node_sets_match_printed_tables(ex):
    g, a, lay = ex
    n = plan_ref.nap_plan(a, lay)
    assert n["N"] == _as_int_dict(g["printed"]["N"]["value"])
    assert triples((x, y, v) for (x, y), v in n["E"].items()) == triples(
        g["printed"]["E"]["value"])
    assert n["T"] == _as_int_dict(g["printed"]["T"]["value"])
    assert n["U"] == _as_int_dict(g["printed"]["U"]["value"])
    assert n["G"] == _as_int_dict(g["printed"]["G"]["value"])


@pytest.mark.parametrize("key,phase", [("I", "INTER"), ("L0", "L0"), ("L1", "L1"), ("L2", "L2")])
def test_messages_match_corrected_tables(ex, key, phase):
    g, a, lay = ex
    n = plan_ref.nap_plan(a, lay)
    assert triples(n["phases"][phase]) == triples(g["corrected"][key]["value"])


def test_corrections_are_exactly_the_documented_errata(ex):
    g, _, _ = ex
    diff = {}
    for key in ("I", "L0", "L1", "L2"):
        printed = set(triples(g["printed"][key]["value"]))
        fixed = set(triples(g["corrected"][key]["value"]))
        diff[key] = (sorted(printed - fixed), sorted(fixed - printed))
    assert diff["I"] == ([(0, 3, (0,)), (1, 5, (0, 1))], [(0, 3, (0, 1)), (1, 5, (0,))])
    assert diff["L0"] == ([], [(1, 0, (1,))])
    assert diff["L1"] == ([(5, 4, (1,))], [(0, 1, (4,)), (5, 4, (0,))])
    assert diff["L2"] == ([], [(2, 3, (2,))])


def test_literal_u_ordering_by_sender_volume_contradicts_table(ex):
    """The mapping rule's text, read with the sender's volume as the U key,
    gives U((0,0)) = {1}; the table prints {2}.  The oracle's reading (the
    receiving node's own volume, opposite direction) gives the table."""
    g, a, lay = ex
    N, E = plan_ref.node_sets(a, lay)
    senders = [m for m in range(3) if 0 in N[m]]
    by_sender_volume = sorted(senders, key=lambda m: (-len(E[(m, 0)]), m))
    assert by_sender_volume[0] == 2          # would map node 2 to (ppn-1, 0) = rank 1
    assert g["printed"]["U"]["value"]["1"] == [1]


def test_totals(ex):
    g, a, lay = ex
    s = plan_ref.standard_plan(a, lay)["phases"]
    n = plan_ref.nap_plan(a, lay)["phases"]
    tot = lambda ph: (len(ph), sum(len(m[2]) for m in ph))  # noqa: E731
    assert tot(s["INTER"]) == (8, 8) and tot(s["L2"]) == (3, 3)
    assert tot(n["INTER"]) == (5, 7)
    assert tot(n["L0"]) == (5, 5) and tot(n["L1"]) == (3, 3) and tot(n["L2"]) == (3, 3)
    assert sum(len(x) for x in plan_ref.ghosts(a, lay)) == 11


@pytest.mark.parametrize("mode", ["standard", "nap"])
def test_vectorised_equals_literal(ex, mode):
    g, a, lay = ex
    lit = plan_ref.plan(a, lay, mode)
    vec = plan_vec.plan(a, 6, 2, mode)
    for ph in plan_ref.PHASES:
        assert arrays_to_triples(vec["phases"][ph]) == triples(lit["phases"][ph])


def test_brute_force_equals_literal(ex):
    g, a, lay = ex
    b = brute.nap_sets(a, 6, 2)
    n = plan_ref.nap_plan(a, lay)
    assert b["E"] == n["E"]
    assert triples((s, d, v) for (s, d), v in b["I"].items()) == triples(n["phases"]["INTER"])
    for key, ph in (("J0", "L0"), ("J1", "L1"), ("J2", "L2")):
        assert triples((s, d, v) for (s, d), v in b[key].items()) == triples(n["phases"][ph])


@pytest.mark.parametrize("mode", ["standard", "nap"])
def test_delivery_and_product(ex, mode):
    g, a, lay = ex
    rng = np.random.default_rng(7)
    a = CSR(a.n, a.rowptr, a.col, rng.integers(-5, 6, size=a.val.size).astype(np.float64))
    v = rng.integers(-9, 10, size=6).astype(np.float64)
    p = plan_ref.plan(a, lay, mode)
    sim = simulate.simulate_standard if mode == "standard" else simulate.simulate_nap
    _, w = sim(a, lay, p, v)
    assert np.array_equal(w, brute.matvec(a, v))
    assert np.array_equal(w, spmv.spmv(a, v))


def test_printed_inter_table_fails_delivery(ex):
    """Planted mistake: with Table example_I as printed (and its local steps),
    the simulation finds a ghost that never arrives."""
    g, a, lay = ex
    p = plan_ref.nap_plan(a, lay)
    bad = {"mode": "nap", "phases": {
        "INTER": triples(g["printed"]["I"]["value"]),
        "L0": triples(g["printed"]["L0"]["value"]),
        "L1": triples(g["printed"]["L1"]["value"]),
        "L2": triples(g["printed"]["L2"]["value"])}}
    with pytest.raises(simulate.DeliveryError):
        simulate.simulate_nap(a, lay, bad, np.arange(6.0))
    simulate.simulate_nap(a, lay, p, np.arange(6.0))


# Every statistic the paper plots per process (section 5), derived by hand
# from the tables of Example 2.1 (the corrected ones for NAP; reading Q9-Q12
# above).  Nodes are {0,1}, {2,3}, {4,5}.
#   standard, D: (1->0)(3->0)(5->0)(4->1)(3->2)(0->3)(1->3)(2->3)(0->4)(2->4)
#     (0->5), one value each.  Inter-node (8): rank 0 sends 3 (to 3, 4, 5);
#     ranks 1, 2, 3, 4, 5 send one each; ranks 0, 3, 4 receive 2 each, 1 and
#     5 one.  Intra-node (3): 1->0, 3->2, 2->3.
#   NAP INTER: (0->3 {0,1}) (1->5 {0}) (2->1 {3}) (3->4 {2}) (4->0 {4,5}):
#     every rank sends and receives at most one message, of at most 2 values.
#   L0: (0->1)(1->0)(2->3)(3->2)(5->4); L1: (0->1)(1->0)(5->4); L2 as the
#     standard intra-node messages: one value each, one per rank.
EXAMPLE_STATS = {
    # (msgs, elems, max_msgs_sent, max_elems_sent, max_msgs_recv, max_elems_recv, max_msg_elems)
    ("standard", "INTER"): (8, 8, 3, 3, 2, 2, 1),
    ("standard", "L2"): (3, 3, 1, 1, 1, 1, 1),
    ("nap", "INTER"): (5, 7, 1, 2, 1, 2, 2),
    ("nap", "L0"): (5, 5, 1, 1, 1, 1, 1),
    ("nap", "L1"): (3, 3, 1, 1, 1, 1, 1),
    ("nap", "L2"): (3, 3, 1, 1, 1, 1, 1),
}
STAT_KEYS = ("msgs", "elems", "max_msgs_sent", "max_elems_sent", "max_msgs_recv",
             "max_elems_recv", "max_msg_elems")


@pytest.mark.parametrize("mode", ["standard", "nap"])
def test_every_phase_statistic_matches_hand_derivation(ex, mode):
    g, a, lay = ex
    vec = plan_vec.plan(a, 6, 2, mode)
    for ph in plan_ref.PHASES:
        want = EXAMPLE_STATS.get((mode, ph), (0,) * 7)
        got = plan_vec.phase_stats(vec["phases"][ph], 6)
        assert tuple(got[k] for k in STAT_KEYS) == want, (mode, ph)


def test_planted_sender_receiver_swap_is_caught(ex):
    """A phase_stats that mixed up senders and receivers would report rank
    0's three inter-node sends as receives; the hand-derived values differ."""
    g, a, lay = ex
    src, dst, ptr, idx = plan_vec.plan(a, 6, 2, "standard")["phases"]["INTER"]
    swapped = plan_vec.phase_stats((dst, src, ptr, idx), 6)
    assert tuple(swapped[k] for k in STAT_KEYS) != EXAMPLE_STATS[("standard", "INTER")]
