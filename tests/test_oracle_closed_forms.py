"""The oracle's plans against closed forms derived by hand for the Laplacian
layouts, and against the special cases of the method.

2D 5-point Laplacian on 64 x 64, n_p = 16, ppn = 4.  Rank t owns grid lines
y = 4t .. 4t+3; it needs line 4t-1 from t-1 and line 4t+4 from t+1, 64
values each.  Standard: 30 messages of 64; the 6 crossing the 3 node
boundaries are inter-node.  NAP: E(n, n+1) is line 16n+15 and E(n+1, n) is
line 16(n+1); node 1 and 2 order their two partners by id (equal volumes),
so the lower partner goes to local 0 (T) and to local 3 (U).  Only the
senders of lines 15, 31, 47 (ranks 0, 5, 9) do not own them: 3 gather
messages; receivers 7, 11, 6, 15, 10 forward to the one rank that uses the
line (rank 3 uses line 16 itself): 5 scatter messages.

3D 7-point Laplacian on 128^3, n_p = 1024, ppn = 16.  Rank t owns 16 lines
of plane z = t div 8; a node holds 2 planes.  Ghosts: 128 per y-neighbour
block, 2048 per z-neighbour block.  Inter-node standard messages cross the 63
node boundaries: 63 * 8 * 2 of 2048.  NAP sends one message per node pair
(126 of 16384).  Interior node a orders partners [a-1, a+1]: local 0 sends
plane 2a, gathered from the 7 other owners; local 1 sends plane 2a+1,
gathered from all 8 owners; local 15 receives from a-1 and scatters to
locals 0-7; local 14 receives from a+1 and scatters to locals 8-13 and 15.
The two end nodes contribute 8+7 gathers and 7+8 scatters.
"""
import numpy as np
import pytest

from oracle import plan_ref, plan_vec
from tests.helpers import arrays_to_triples, triples
from workloads import config, kkt_like, laplacian_2d, laplacian_3d, random_pattern


def _tot(phase):
    src, dst, ptr, idx = phase
    return (int(src.size), int(ptr[-1]))


def test_laplace2d_closed_forms():
    a = laplacian_2d(64, 64)
    assert a.nnz == 5 * 4096 - 4 * 64
    s = plan_vec.standard_plan(a, 16, 4)
    n = plan_vec.nap_plan(a, 16, 4)
    assert s["ghost_t"].size == 14 * 128 + 2 * 64
    assert _tot(s["phases"]["INTER"]) == (6, 384)
    assert _tot(s["phases"]["L2"]) == (24, 1536)
    assert _tot(n["phases"]["INTER"]) == (6, 384)
    assert _tot(n["phases"]["L0"]) == (3, 192)
    assert _tot(n["phases"]["L1"]) == (5, 320)
    assert _tot(n["phases"]["L2"]) == (24, 1536)
    inter = arrays_to_triples(n["phases"]["INTER"])
    assert [(x, y) for x, y, _ in inter] == [(0, 7), (4, 3), (5, 11), (8, 6), (9, 15), (12, 10)]
    assert [(x, y) for x, y, _ in arrays_to_triples(n["phases"]["L0"])] == [(3, 0), (7, 5), (11, 9)]
    assert [(x, y) for x, y, _ in arrays_to_triples(n["phases"]["L1"])] == [
        (6, 7), (7, 4), (10, 11), (11, 8), (15, 12)]
    # the literal oracle agrees message by message
    lay = plan_ref.Layout(a.n, 16, 4)
    lit = plan_ref.nap_plan(a, lay)
    for ph in plan_ref.PHASES:
        assert arrays_to_triples(n["phases"][ph]) == triples(lit["phases"][ph])


def test_laplace3d_closed_forms():
    a = laplacian_3d(128, 128, 128)
    assert a.nnz == 7 * 128 ** 3 - 6 * 128 ** 2
    s = plan_vec.standard_plan(a, 1024, 16)
    n = plan_vec.nap_plan(a, 1024, 16)
    g = s["ghost_t"].size
    assert g == 128 * 7 * 2 * 128 + 127 * 8 * 2 * 2048
    assert _tot(s["phases"]["INTER"]) == (63 * 8 * 2, 63 * 8 * 2 * 2048)
    assert _tot(s["phases"]["L2"]) == (7 * 2 * 128 + 64 * 8 * 2, 7 * 2 * 128 * 128 + 64 * 8 * 2 * 2048)
    assert _tot(n["phases"]["INTER"]) == (126, 126 * 16384)
    assert _tot(n["phases"]["L0"]) == (62 * 15 + 8 + 7, (62 * 15 + 15) * 2048)
    assert _tot(n["phases"]["L1"]) == (62 * 15 + 7 + 8, (62 * 15 + 15) * 2048)
    assert _tot(n["phases"]["L2"]) == _tot(s["phases"]["L2"])
    st = plan_vec.phase_stats(s["phases"]["INTER"], 1024)
    nt = plan_vec.phase_stats(n["phases"]["INTER"], 1024)
    assert st["max_elems_sent"] == 2048 and nt["max_elems_sent"] == 16384


def test_ppn_one_nap_equals_standard():
    """One process per node: every exchange is inter-node, E(n, m) = D(n, m),
    and the local steps are empty."""
    a = random_pattern(50, 0.1, seed=11)
    for n_p in (1, 3, 7):
        s = plan_vec.standard_plan(a, n_p, 1)
        n = plan_vec.nap_plan(a, n_p, 1)
        assert arrays_to_triples(n["phases"]["INTER"]) == arrays_to_triples(s["phases"]["INTER"])
        for ph in ("L0", "L1", "L2"):
            assert _tot(n["phases"][ph]) == (0, 0)
        assert _tot(s["phases"]["L2"]) == (0, 0)


def test_single_node_everything_local():
    """ppn = n_p: no inter-node traffic; the fully local step equals the
    standard messages."""
    a = laplacian_2d(64, 64)
    s = plan_vec.standard_plan(a, 16, 16)
    n = plan_vec.nap_plan(a, 16, 16)
    assert _tot(s["phases"]["INTER"]) == (0, 0) and _tot(n["phases"]["INTER"]) == (0, 0)
    assert _tot(s["phases"]["L2"]) == (30, 1920)
    assert arrays_to_triples(n["phases"]["L2"]) == arrays_to_triples(s["phases"]["L2"])
    a1 = plan_vec.standard_plan(a, 16, 1)
    assert _tot(a1["phases"]["INTER"]) == (30, 1920)


def test_single_process_no_messages():
    a = random_pattern(30, 0.2, seed=2)
    for mode in ("standard", "nap"):
        p = plan_vec.plan(a, 1, 1, mode)
        assert p["ghost_t"].size == 0
        for ph in plan_ref.PHASES:
            assert _tot(p["phases"][ph]) == (0, 0)


@pytest.mark.parametrize("maker", [
    lambda: config(1), lambda: config(2, scale=3), lambda: config(3, scale=6),
    lambda: config(4, scale=4)])
def test_invariants(maker):
    """Invariants the paper states for NAPSpMV: no more inter-node messages or
    elements than standard; the fully local step equals standard's
    intra-node messages; E(n, m) is the union of D(r, t) over the node pair
    and is sent in one message."""
    wl = maker()
    a, n_p, ppn = wl.csr, wl.n_p, wl.ppn
    s = plan_vec.standard_plan(a, n_p, ppn, wl.row_starts)
    n = plan_vec.nap_plan(a, n_p, ppn, wl.row_starts)
    si, ni = _tot(s["phases"]["INTER"]), _tot(n["phases"]["INTER"])
    assert ni[0] <= si[0] and ni[1] <= si[1]
    assert arrays_to_triples(n["phases"]["L2"]) == arrays_to_triples(s["phases"]["L2"])
    starts = s["starts"]
    node = lambda r: r // ppn  # noqa: E731
    union = {}
    for r, t, idx in arrays_to_triples(s["phases"]["INTER"]):
        union.setdefault((node(r), node(t)), set()).update(idx)
    got = {}
    for x, y, idx in arrays_to_triples(n["phases"]["INTER"]):
        key = (node(x), node(y))
        assert key not in got                       # one message per node pair
        got[key] = set(idx)
    assert got == union
    # every ghost of every rank is delivered exactly once by the NAP phases
    t, j = n["ghost_t"], n["ghost_j"]
    own = plan_vec.owner(starts, j)
    on = node(own) == node(t)
    l2 = {(y, int(i)) for x, y, idx in arrays_to_triples(n["phases"]["L2"]) for i in idx}
    l1 = {(y, int(i)) for x, y, idx in arrays_to_triples(n["phases"]["L1"]) for i in idx}
    rec = {}
    for x, y, idx in arrays_to_triples(n["phases"]["INTER"]):
        for i in idx:
            rec[(node(y), int(i))] = y
    for tt, jj, o in zip(t.tolist(), j.tolist(), on.tolist()):
        if o:
            assert (tt, jj) in l2
        else:
            q = rec[(node(tt), jj)]
            assert (q == tt) != ((tt, jj) in l1)


STAT_KEYS = ("msgs", "elems", "max_msgs_sent", "max_elems_sent", "max_msgs_recv",
             "max_elems_recv", "max_msg_elems")


def _stats(phase, n_p):
    st = plan_vec.phase_stats(phase, n_p)
    return tuple(st[k] for k in STAT_KEYS)


def test_laplace2d_per_process_statistics():
    """All seven statistics per phase (section 5 plots the per-process ones).
    Standard inter-node: ranks 3, 4, 7, 8, 11, 12 each send one line to the
    neighbour across a node boundary and receive one.  Intra-node: the two
    middle ranks of a node exchange a line with both neighbours (2 messages,
    128 values each way).  NAP: every INTER sender, L0 and L1 rank moves
    exactly one line (the message lists are in test_laplace2d_closed_forms)."""
    a = laplacian_2d(64, 64)
    s = plan_vec.standard_plan(a, 16, 4)["phases"]
    n = plan_vec.nap_plan(a, 16, 4)["phases"]
    assert _stats(s["INTER"], 16) == (6, 384, 1, 64, 1, 64, 64)
    assert _stats(s["L2"], 16) == (24, 1536, 2, 128, 2, 128, 64)
    assert _stats(n["INTER"], 16) == (6, 384, 1, 64, 1, 64, 64)
    assert _stats(n["L0"], 16) == (3, 192, 1, 64, 1, 64, 64)
    assert _stats(n["L1"], 16) == (5, 320, 1, 64, 1, 64, 64)
    assert _stats(n["L2"], 16) == _stats(s["L2"], 16)


def test_laplace3d_per_process_statistics():
    """Rank t owns y-block t mod 8 (16 lines) of plane t div 8; a node holds
    planes 2a and 2a+1 (locals 0-7 and 8-15).
    Standard inter-node: a rank of plane 2a+1 sends its block up to plane
    2a+2, a rank of plane 2a down to 2a-1: one message of 2048 each way.
    Standard intra-node: an interior y-block sends a line (128) to each y
    neighbour and its block (2048) to the other plane of its node: 3
    messages, 2304 values, sent and received alike.
    NAP INTER: local 0 sends plane 2a to node a-1 and local 1 plane 2a+1 to
    node a+1 (equal volumes, lower node id first); local 15 receives from
    a-1 and local 14 from a+1: one message of 16384 per rank at most.
    L0: local 1 gathers plane 2a+1 from its 8 owners (8 x 2048 received),
    local 0 plane 2a from the 7 others; every owner sends one block.
    L1: local 15 forwards plane 2a-1 to locals 0-7 (8 x 2048 sent), local 14
    plane 2a+2 to locals 8-13 and 15; every user receives one block."""
    a = laplacian_3d(128, 128, 128)
    s = plan_vec.standard_plan(a, 1024, 16)["phases"]
    n = plan_vec.nap_plan(a, 1024, 16)["phases"]
    assert _stats(s["INTER"], 1024) == (1008, 1008 * 2048, 1, 2048, 1, 2048, 2048)
    intra = (7 * 2 * 128 + 64 * 8 * 2, 7 * 2 * 128 * 128 + 64 * 8 * 2 * 2048)
    assert _stats(s["L2"], 1024) == intra + (3, 2304, 3, 2304, 2048)
    assert _stats(n["INTER"], 1024) == (126, 126 * 16384, 1, 16384, 1, 16384, 16384)
    assert _stats(n["L0"], 1024) == (945, 945 * 2048, 1, 2048, 8, 16384, 2048)
    assert _stats(n["L1"], 1024) == (945, 945 * 2048, 8, 16384, 1, 2048, 2048)
    assert _stats(n["L2"], 1024) == _stats(s["L2"], 1024)


def test_planted_swap_caught_by_laplace3d_pins():
    """A sender/receiver mix-up in phase_stats turns L0's 8 gathered blocks
    per sender into 8 sends per owner; the hand-derived pins catch it."""
    a = laplacian_3d(128, 128, 128)
    src, dst, ptr, idx = plan_vec.nap_plan(a, 1024, 16)["phases"]["L0"]
    assert _stats((dst, src, ptr, idx), 1024) != (945, 945 * 2048, 1, 2048, 8, 16384, 2048)
