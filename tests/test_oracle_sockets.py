"""The oracle's third hierarchy level: sockets of pps consecutive ranks inside
a node route the three intra-node steps the way section 4 routes inter-node
messages (reading in the module docstring of ``oracle.plan_ref``; section 6
names on-socket and off-socket intra-node messages as future work).

Pins: a hand-derived example, three independent evaluations (literal sets,
NumPy, quantifier brute force with a lexsort mapping) agreeing, the two
reductions to the two-level plan (one socket per node, one rank per socket),
invariants (one message per socket pair carrying the union of the pair's
off-socket messages, never more off-socket messages or values than the
two-level plan), exactly-once delivery with planted mistakes caught, and a
closed form on the 3D Laplacian with one plane per socket.
"""
import numpy as np
import pytest

from oracle import brute, plan_ref, plan_vec, simulate, spmv
from tests.helpers import arrays_to_triples, csr_from_rows, triples
from workloads import CSR, laplacian_3d, random_pattern


def _hand_example():
    """One node of 4 ranks (2 rows each), sockets {0, 1} and {2, 3}.
    Off-process entries: row 4 (rank 2) uses v0, v2; row 6 (rank 3) uses
    v0, v3; row 0 (rank 0) uses v6; row 2 (rank 1) uses v7; row 3 (rank 1)
    uses v1."""
    rows = [[0, 6], [1], [2, 7], [1, 3], [0, 2, 4], [5], [0, 3, 6], [7]]
    return csr_from_rows(rows)


def test_hand_derived_single_node():
    """Fully local step: 0->1 {1} stays on socket 0.  Socket 0 -> 1 carries
    F = {0, 2, 3} (0->2 {0}, 0->3 {0}, 1->2 {2}, 1->3 {3}: v0 once);
    socket 1 -> 0 carries {6, 7} (3->0 {6}, 3->1 {7}).  Each socket has one
    partner: sender = its first rank, receiver = its last rank (pps-1), so
    0 sends to 3 and 2 sends to 1.  Rank 1 hands {2, 3} to rank 0, rank 3
    hands {6, 7} to rank 2; rank 3 keeps v3 and forwards {0, 2} to rank 2;
    rank 1 keeps v7 and forwards {6} to rank 0."""
    a = _hand_example()
    lay = plan_ref.Layout(8, 4, 4)
    p = plan_ref.socket_plan(a, lay, 2)["phases"]
    assert triples(p["L2"]) == [(0, 1, (1,)), (0, 2, (0,)), (0, 3, (0,)), (1, 2, (2,)),
                                (1, 3, (3,)), (3, 0, (6,)), (3, 1, (7,))]
    assert triples(p["L2_on"]) == [(0, 1, (1,))]
    assert triples(p["L2_cross"]) == [(0, 3, (0, 2, 3)), (2, 1, (6, 7))]
    assert triples(p["L2_gather"]) == [(1, 0, (2, 3)), (3, 2, (6, 7))]
    assert triples(p["L2_scatter"]) == [(1, 0, (6,)), (3, 2, (0, 2))]
    for ph in ("L0", "L1"):
        for part in plan_ref.SOCKET_PARTS:
            assert p[f"{ph}_{part}"] == []
    # six off-socket messages of 6 values become two of 5
    v = np.arange(8.0) - 3.0
    _, w = simulate.simulate_nap(a, lay, plan_ref.socket_plan(a, lay, 2), v)
    assert np.array_equal(w, spmv.spmv_split(a, v, 4))


CASES = [(60, 8, 4, 2, 1), (90, 12, 6, 2, 2), (90, 12, 6, 3, 3), (120, 16, 8, 2, 4),
         (64, 8, 8, 4, 5), (97, 16, 4, 2, 6), (130, 16, 8, 4, 7)]


@pytest.mark.parametrize("n,n_p,ppn,pps,seed", CASES)
def test_three_routes_agree_and_deliver(n, n_p, ppn, pps, seed):
    a = random_pattern(n, 0.08, seed=seed, empty_rows=2, duplicates=3)
    lay = plan_ref.Layout(n, n_p, ppn)
    lit = plan_ref.socket_plan(a, lay, pps)
    vec = plan_vec.socket_plan(a, n_p, ppn, pps)
    br = brute.socket_sets(a, n_p, ppn, pps)
    for ph in plan_ref.SOCKET_PHASES:
        assert arrays_to_triples(vec["phases"][ph]) == triples(lit["phases"][ph]), ph
        step = {"L0": "J0", "L1": "J1", "L2": "J2"}[ph[:2]]
        got = triples((s, d, v) for (s, d), v in br[step][ph[3:]].items())
        assert got == triples(lit["phases"][ph]), ph
    v = np.random.default_rng(seed).integers(-9, 10, n).astype(np.float64)
    _, w = simulate.simulate_nap(a, lay, lit, v)
    assert np.array_equal(w, spmv.spmv_split(a, v, n_p))


def test_explicit_row_starts():
    a = random_pattern(80, 0.09, seed=21)
    starts = [0, 3, 10, 20, 26, 40, 41, 60, 80]
    lay = plan_ref.Layout(80, 8, 4, row_starts=starts)
    lit = plan_ref.socket_plan(a, lay, 2)
    vec = plan_vec.socket_plan(a, 8, 4, 2, given_starts=starts)
    for ph in plan_ref.SOCKET_PHASES:
        assert arrays_to_triples(vec["phases"][ph]) == triples(lit["phases"][ph]), ph
    simulate.simulate_nap(a, lay, lit, np.arange(80.0))


@pytest.mark.parametrize("seed", [1, 2])
def test_reductions_to_the_two_level_plan(seed):
    """One socket per node: every intra-node message stays on its socket.
    One rank per socket: every socket pair is a rank pair, its sender and
    receiver are those ranks, and nothing is gathered or forwarded."""
    a = random_pattern(96, 0.08, seed=seed)
    lay = plan_ref.Layout(96, 12, 4)
    base = plan_ref.nap_plan(a, lay)["phases"]
    whole = plan_ref.socket_plan(a, lay, 4)["phases"]
    single = plan_ref.socket_plan(a, lay, 1)["phases"]
    for ph in ("L0", "L1", "L2"):
        assert triples(whole[f"{ph}_on"]) == triples(base[ph])
        assert triples(single[f"{ph}_cross"]) == triples(base[ph])
        for part in ("gather", "cross", "scatter"):
            assert whole[f"{ph}_{part}"] == []
        for part in ("on", "gather", "scatter"):
            assert single[f"{ph}_{part}"] == []


@pytest.mark.parametrize("n,n_p,ppn,pps,seed", CASES)
def test_invariants(n, n_p, ppn, pps, seed):
    """Per socket pair one cross message, carrying exactly the union of the
    two-level step's off-socket messages between the two sockets; hence
    never more off-socket messages or values than the two-level plan.  The
    on-socket part is the two-level step's on-socket messages unchanged, and
    gather and scatter messages never leave a socket."""
    a = random_pattern(n, 0.08, seed=seed)
    lay = plan_ref.Layout(n, n_p, ppn)
    p = plan_ref.socket_plan(a, lay, pps)["phases"]
    sock = lambda r: r // pps  # noqa: E731
    for ph in ("L0", "L1", "L2"):
        base = triples(p[ph])
        off = [m for m in base if sock(m[0]) != sock(m[1])]
        union = {}
        for x, y, idx in off:
            union.setdefault((sock(x), sock(y)), set()).update(idx)
        cross = {}
        for q, r, idx in triples(p[f"{ph}_cross"]):
            key = (sock(q), sock(r))
            assert key not in cross and lay.node(q) == lay.node(r)
            cross[key] = set(idx)
        assert cross == union
        assert len(cross) <= len(off)
        assert sum(len(x) for x in cross.values()) <= sum(len(m[2]) for m in off)
        assert triples(p[f"{ph}_on"]) == [m for m in base if sock(m[0]) == sock(m[1])]
        for part in ("gather", "scatter"):
            assert all(sock(x) == sock(y) for x, y, _ in triples(p[f"{ph}_{part}"]))


def test_planted_route_mistakes_fail_delivery():
    a = random_pattern(90, 0.08, seed=2)
    lay = plan_ref.Layout(90, 12, 6)
    v = np.arange(90.0)
    good = plan_ref.socket_plan(a, lay, 2)
    simulate.simulate_nap(a, lay, good, v)
    for ph in ("L0_scatter", "L1_gather", "L2_cross", "L2_scatter", "L1_on"):
        assert good["phases"][ph], ph
        bad = dict(good, phases=dict(good["phases"]))
        bad["phases"][ph] = good["phases"][ph][1:]          # one message lost
        with pytest.raises(simulate.DeliveryError):
            simulate.simulate_nap(a, lay, bad, v)
    # a cross message sent by the receiver instead of the sender
    bad = dict(good, phases=dict(good["phases"]))
    q, r, idx = good["phases"]["L2_cross"][0]
    bad["phases"]["L2_cross"] = [(r, q, idx)] + good["phases"]["L2_cross"][1:]
    with pytest.raises(simulate.DeliveryError):
        simulate.simulate_nap(a, lay, bad, v)


def _tot(phase):
    src, dst, ptr, idx = phase
    return (int(src.size), int(ptr[-1]))


def test_laplace3d_one_plane_per_socket_closed_form():
    """128^3, n_p 1024, ppn 16, pps 8: socket 0 of node a is plane 2a
    (locals 0-7), socket 1 plane 2a+1 (locals 8-15); each socket's one
    partner is sent by its first rank and received by its last (locals 0/8
    send, 7/15 receive).
    Fully local step: the y-neighbour lines stay on their socket (1792 of
    128); the 16 z-messages of 2048 between the two planes of a node become
    one cross message of 16384 each way (128), with 7 gathers of 2048 into
    the sender and 7 forwards of 2048 from the receiver (896 each).
    on_node -> off_node: local 0 gathers plane 2a on its socket (7 of 2048,
    on-socket); local 1 needs plane 2a+1 from socket 1: locals 9-15 hand
    their blocks to local 8 (7 of 2048), 8 sends the plane to 7 (16384), 7
    forwards it to 1 (16384).  Node 0 (partner 1 only) routes plane 1 to its
    local 0 the same way; node 63 gathers plane 126 on socket 0 only.
    off_node -> on_node: local 15 (socket 1) received plane 2a-1 for plane
    2a: it hands it to 8 (16384), 8 sends to 7, 7 keeps block 7 and
    forwards 7 blocks of 2048; local 14's plane 2a+2 stays on socket 1 (7
    of 2048).  Node 0 forwards plane 2 on socket 1 only; node 63 routes
    plane 125 across."""
    a = laplacian_3d(128, 128, 128)
    p = plan_vec.socket_plan(a, 1024, 16, 8)["phases"]
    assert _tot(p["L2_on"]) == (1792, 1792 * 128)
    assert _tot(p["L2_gather"]) == (896, 896 * 2048)
    assert _tot(p["L2_cross"]) == (128, 128 * 16384)
    assert _tot(p["L2_scatter"]) == (896, 896 * 2048)
    assert _tot(p["L0_on"]) == (441, 441 * 2048)
    assert _tot(p["L0_gather"]) == (441, 441 * 2048)
    assert _tot(p["L0_cross"]) == (63, 63 * 16384)
    assert _tot(p["L0_scatter"]) == (63, 63 * 16384)
    assert _tot(p["L1_on"]) == (441, 441 * 2048)
    assert _tot(p["L1_gather"]) == (63, 63 * 16384)
    assert _tot(p["L1_cross"]) == (63, 63 * 16384)
    assert _tot(p["L1_scatter"]) == (441, 441 * 2048)
    st = plan_vec.phase_stats(p["L2_cross"], 1024)
    assert (st["max_msgs_sent"], st["max_elems_sent"], st["max_msgs_recv"]) == (1, 16384, 1)
    # the z-exchange between the planes of a node: 8 off-socket messages
    # each way before, one after
    two = plan_vec.phase_stats(p["L2"], 1024)
    assert two["msgs"] == 2816 and two["msgs"] - 1792 == 64 * 16
