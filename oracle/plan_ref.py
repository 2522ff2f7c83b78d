"""Literal, set-based evaluation of the communication sets of the standard SpMV
(section 2.1) and of the node-aware parallel SpMV, NAPSpMV (section 4).

Test infrastructure (see the package docstring): plain Python sets, one stored
entry at a time, for tiny and small matrices only.

Notation follows the paper.  Rank ``r`` is the pair ``(p, n)`` with local
number ``p = r mod ppn`` and node ``n = floor(r / ppn)`` (section 2, SMP-style
ordering).  ``R(r)`` is the contiguous row block of rank ``r``.  A stored entry
``(i, j)`` of the CSR pattern is a nonzero ``A_ij`` (reading: structural; an
explicitly stored zero counts, since the sets describe communication and do
not depend on values).

Readings taken where the paper is silent, garbled or at odds with itself:

* Remainder rows.  The even partition ``R(r) = {floor(N/n_p) r, ...,
  floor(N/n_p)(r+1) - 1}`` leaves ``N mod n_p`` rows unassigned; the last
  rank takes them.  Explicit block boundaries may be given instead.
* ``D(r, t)`` and ``E(n, m)`` are written as sets of row indices ``i``, but
  the worked example's tables list the column ``j`` (the vector index owned by
  the sender); they are read as sets of ``j``.  The volume ``|D(n, m)|`` used
  by the mapping rule is read as ``|E(n, m)|``.
* Mapping of partner nodes to local processes (rule stated after the
  definitions of T and U).  The partners of node ``n`` are ordered by
  ``|E(n, m)|`` descending, ties by ascending node id; the k-th partner goes
  to local process ``k mod ppn`` (T).  The nodes that send to ``n`` are
  ordered by the same key (what ``n`` sends to them, 0 if nothing), ties by
  ascending id, and the k-th goes to local process ``ppn - 1 - (k mod ppn)``
  (U: the opposite ordering).  This reproduces every entry of the worked
  example's T/U table; ordering U by the sender's own volume does not.  When a
  node has fewer partners than ppn, no partner is split over several
  processes (the worked example's table does not split).
* ``J`` of the on_node -> off_node step (its quantifier is garbled): the
  indices owned by ``(p, n)`` that appear in any inter-node message sent by
  ``(s, n)``, for ``s != p``.
* No process sends a message to itself, and messages are deduplicated within
  one (phase, source, destination) pair, not across phases: the fully local
  step carries every on-node ghost even when the same value also travels in
  the on_node -> off_node step.
* The off_node -> on_node step forwards values received in the inter-node
  step (algorithm NAPSpMV passes ``v|R`` there; the received buffer is
  meant), and the receiving process uses its own received values directly.

Variants (none is the default; each leaves every ghost value and w unchanged):

* ``owner_map``: the other mapping section 4.1 names but does not explore:
  partner node m of n is sent by the process of n that owns the most indices
  of E(n, m) (ties: the lowest local number).  U is unchanged.
* ``split``: the rule section 4.1 states for a node with fewer partners than
  processes per node, where one partner is spread over several local
  processes so that every process takes part (the worked example's table
  does not do this, hence not the default).  Read as: the i-th of k < ppn
  partners (T order) is sent by local processes i, i + k, i + 2k, ... < ppn,
  E(n, m) cut into that many contiguous pieces of near-equal length in index
  order, piece c sent by the c-th of them; on the receiving side the i'-th
  of k' < ppn senders (U order) is received by local processes ppn-1-i',
  ppn-1-i'-k', ..., and piece c goes to the (c mod count)-th of those.  A
  node with at least ppn partners (senders) keeps the mapping's choice.
* ``dedup``: not in the paper; the fully local step does not carry an index
  that the on_node -> off_node step already carries between the same two
  processes (the receiving process uses that copy for its own product too).
  This is not what Table example_L2 prints either (it keeps (1,1) -> (0,1):
  {3}, which that step also carries).
* ``three_way``: no change to any set; the product is summed in three parts
  as algorithm NAPSpMV writes it (``spmv.spmv_split3``).

A third hierarchy level (section 6 names splitting intra-node messages into
on-socket and off-socket ones as future work, and the introduction says
socket information could be used the way node information is): sockets of
``pps`` consecutive ranks inside a node.  Reading (``socket_plan``): each of
the three intra-node steps keeps its messages whose two ranks share a socket
(``on``), and routes the others the way section 4 routes inter-node messages,
one level down: per ordered socket pair (s, s') of a node, F(s, s') is the
sorted union of the indices its off-socket messages carry from s to s'
(deduplicated); one process of s sends F(s, s') to one process of s'
(``cross``), chosen by the node-level mapping rule applied to the sockets of
the node (partners of s by |F(s, .)| descending, ties by ascending socket,
the k-th sent by the k mod pps-th process of s; senders to s by the same key,
the k-th received by process pps-1-(k mod pps) of s); the holder of each
index (its owner for the on_node -> off_node and fully local steps, the
inter-node receiver for the off_node -> on_node step; unique within a node)
hands it to the socket sender first (``gather``, deduplicated per pair), and
the socket receiver forwards it to every other process of s' whose message
carried it (``scatter``), using its own values directly.  One socket per node
(pps = ppn) or one process per socket (pps = 1) leaves the two-level plan.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

PHASES = ("INTER", "L0", "L1", "L2")
VARIANTS = frozenset({"owner_map", "dedup", "split", "three_way"})
SOCKET_PARTS = ("on", "gather", "cross", "scatter")
SOCKET_PHASES = tuple(f"{ph}_{part}" for ph in ("L0", "L1", "L2") for part in SOCKET_PARTS)


class Layout:
    """Processes, nodes and row blocks (section 2).  ``strided=True`` gives
    the strided partition of section 5 instead: row r on process
    r mod n_p."""

    def __init__(self, n: int, n_p: int, ppn: int, row_starts=None, strided: bool = False):
        if n_p < 1 or ppn < 1 or n_p % ppn != 0:
            raise ValueError("need n_p >= 1, ppn >= 1 and ppn dividing n_p")
        if n < n_p:
            raise ValueError("need at least one row per process")
        self.n, self.n_p, self.ppn = int(n), int(n_p), int(ppn)
        self.n_nodes = self.n_p // self.ppn
        self.strided = bool(strided)
        if strided:
            if row_starts is not None:
                raise ValueError("a strided partition takes no row_starts")
            self.starts = None
            self._owner = np.arange(self.n, dtype=np.int64) % self.n_p
            return
        if row_starts is None:
            b = self.n // self.n_p
            starts = [b * r for r in range(self.n_p)] + [self.n]
        else:
            starts = [int(x) for x in row_starts]
            if (len(starts) != self.n_p + 1 or starts[0] != 0 or starts[-1] != self.n
                    or any(starts[r + 1] <= starts[r] for r in range(self.n_p))):
                raise ValueError("row_starts must rise strictly from 0 to N")
        self.starts = starts
        self._owner = np.empty(self.n, dtype=np.int64)
        for r in range(self.n_p):
            self._owner[starts[r]:starts[r + 1]] = r

    def R(self, r: int) -> range:
        if self.strided:
            return range(r, self.n, self.n_p)
        return range(self.starts[r], self.starts[r + 1])

    def owner(self, j: int) -> int:
        """The rank r with j in R(r)."""
        return int(self._owner[j])

    def node(self, r: int) -> int:
        return r // self.ppn

    def local(self, r: int) -> int:
        return r % self.ppn

    def rank(self, p: int, n: int) -> int:
        return n * self.ppn + p


def stored_entries(csr):
    """Yield (i, j) for every stored entry, in stored order."""
    rp, col = csr.rowptr, csr.col
    for i in range(csr.n):
        for k in range(int(rp[i]), int(rp[i + 1])):
            yield i, int(col[k])


def ghosts(csr, lay: Layout):
    """gh(t): sorted off-process columns of rank t (the columns of the
    off_process block)."""
    gh = [set() for _ in range(lay.n_p)]
    for i, j in stored_entries(csr):
        t = lay.owner(i)
        if lay.owner(j) != t:
            gh[t].add(j)
    return [sorted(s) for s in gh]


def _canon(sets: dict) -> list:
    """{(src, dst): set} -> [(src, dst, sorted tuple)] sorted by (src, dst)."""
    return [(s, d, tuple(sorted(v))) for (s, d), v in sorted(sets.items()) if v]


def standard_plan(csr, lay: Layout) -> dict:
    """P(r) and D(r, t) of section 2.1, each message classed inter-node or
    intra-node by the nodes of its two ranks."""
    P = defaultdict(set)
    D = defaultdict(set)
    for i, j in stored_entries(csr):
        t, r = lay.owner(i), lay.owner(j)
        if r != t:
            P[r].add(t)
            D[(r, t)].add(j)
    msgs = _canon(D)
    inter = [m for m in msgs if lay.node(m[0]) != lay.node(m[1])]
    intra = [m for m in msgs if lay.node(m[0]) == lay.node(m[1])]
    return {
        "mode": "standard",
        "P": {r: sorted(P[r]) for r in range(lay.n_p)},
        "D": {k: sorted(v) for k, v in D.items()},
        "phases": {"INTER": inter, "L0": [], "L1": [], "L2": intra},
    }


def node_sets(csr, lay: Layout):
    """N(n) and E(n, m) of section 4.1."""
    E = defaultdict(set)
    for i, j in stored_entries(csr):
        m, n = lay.node(lay.owner(i)), lay.node(lay.owner(j))
        if n != m:
            E[(n, m)].add(j)
    N = {n: sorted(m for (a, m) in E if a == n) for n in range(lay.n_nodes)}
    return N, {k: sorted(v) for k, v in E.items()}


def mapping(lay: Layout, N: dict, E: dict, owner_map: bool = False):
    """T((p, n)) and U((p, n)) of section 4.1 under the mapping rule stated
    there (see the module docstring for the reading and the variant).

    Returns (T, U, t_rank, u_rank): T and U map rank -> sorted node list;
    t_rank[(n, m)] is the rank on n sending to node m, u_rank[(n, m)] the rank
    on m receiving from node n.
    """
    def order(n, partners):
        return sorted(partners, key=lambda m: (-len(E.get((n, m), ())), m))

    T = {r: [] for r in range(lay.n_p)}
    U = {r: [] for r in range(lay.n_p)}
    t_rank, u_rank = {}, {}
    for n in range(lay.n_nodes):
        for k, m in enumerate(order(n, N[n])):
            if owner_map:
                held = [sum(1 for j in E[(n, m)] if lay.owner(j) == lay.rank(p, n))
                        for p in range(lay.ppn)]
                r = lay.rank(held.index(max(held)), n)
            else:
                r = lay.rank(k % lay.ppn, n)
            T[r].append(m)
            t_rank[(n, m)] = r
        senders = [m for m in range(lay.n_nodes) if n in N[m]]
        for k, m in enumerate(order(n, senders)):
            r = lay.rank(lay.ppn - 1 - (k % lay.ppn), n)
            U[r].append(m)
            u_rank[(m, n)] = r
    T = {r: sorted(v) for r, v in T.items()}
    U = {r: sorted(v) for r, v in U.items()}
    return T, U, t_rank, u_rank


def split_messages(lay: Layout, N: dict, E: dict, t_rank: dict, u_rank: dict):
    """The ``split`` variant: {(sender, receiver): piece of E(n, m)}, each
    piece sent in its own message.  Only a node with fewer partners (or
    senders) than processes splits; elsewhere the sender and receiver are
    those of the mapping (``t_rank``, ``u_rank``)."""
    def order(n, partners):
        return sorted(partners, key=lambda m: (-len(E.get((n, m), ())), m))

    senders_of, receivers_of = {}, {}
    for n in range(lay.n_nodes):
        part = order(n, N[n])
        k = len(part)
        for i, m in enumerate(part):
            senders_of[(n, m)] = ([lay.rank(p, n) for p in range(i, lay.ppn, k)]
                                  if k < lay.ppn else [t_rank[(n, m)]])
        snd = order(n, [m for m in range(lay.n_nodes) if n in N[m]])
        k2 = len(snd)
        for i, m in enumerate(snd):
            receivers_of[(m, n)] = ([lay.rank(p, n) for p in range(lay.ppn - 1 - i, -1, -k2)]
                                    if k2 < lay.ppn else [u_rank[(m, n)]])
    msgs = {}
    for (n, m), idx in E.items():
        s_list, r_list = senders_of[(n, m)], receivers_of[(n, m)]
        c = len(s_list)
        L = len(idx)
        for piece in range(c):
            part = idx[piece * L // c:(piece + 1) * L // c]
            if part:
                msgs[(s_list[piece], r_list[piece % len(r_list)])] = set(part)
    return msgs


def nap_plan(csr, lay: Layout, variant=()) -> dict:
    """Every set of section 4: N, E, T, U, G, I and the three local steps,
    under the default readings or the named variants."""
    variant = set(variant)
    if variant - VARIANTS:
        raise ValueError(f"unknown variant(s) {sorted(variant - VARIANTS)}")
    N, E = node_sets(csr, lay)
    T, U, t_rank, u_rank = mapping(lay, N, E, owner_map="owner_map" in variant)

    # G((p, n)) = {(q, m) | m in T((p, n)), n in U((q, m))};  I = E(n, m).
    G = defaultdict(set)
    I = {}
    if "split" in variant:
        I = split_messages(lay, N, E, t_rank, u_rank)
        for (s, q) in I:
            G[s].add(q)
    else:
        for s in range(lay.n_p):
            n = lay.node(s)
            for m in T[s]:
                for q in (lay.rank(x, m) for x in range(lay.ppn)):
                    if n in U[q]:
                        G[s].add(q)
                        I[(s, q)] = set(E[(n, m)])

    # on_node -> off_node: owners hand their values to the inter-node sender.
    J0 = defaultdict(set)
    for (s, q), idx in I.items():
        for j in idx:
            p = lay.owner(j)
            if p != s:
                J0[(p, s)].add(j)

    # off_node -> on_node: the receiver forwards to the processes that use a value.
    J1 = defaultdict(set)
    recv_of = {}
    for (s, q), idx in I.items():
        for j in idx:
            recv_of[j, lay.node(q)] = q
    for i, j in stored_entries(csr):
        t = lay.owner(i)
        q = recv_of.get((j, lay.node(t)))
        if q is not None and q != t and lay.node(lay.owner(j)) != lay.node(t):
            J1[(q, t)].add(j)

    # on_node -> on_node: direct messages between processes of one node.
    J2 = defaultdict(set)
    for i, j in stored_entries(csr):
        t, r = lay.owner(i), lay.owner(j)
        if r != t and lay.node(r) == lay.node(t):
            J2[(r, t)].add(j)
    if "dedup" in variant:
        for key in list(J2):
            J2[key] -= J0.get(key, set())

    return {
        "mode": "nap", "variant": sorted(variant),
        "N": N, "E": E, "T": T, "U": U,
        "t_rank": t_rank, "u_rank": u_rank,
        "G": {s: sorted(G[s]) for s in range(lay.n_p)},
        "I": {k: sorted(v) for k, v in I.items()},
        "phases": {"INTER": _canon(I), "L0": _canon(J0), "L1": _canon(J1),
                   "L2": _canon(J2)},
    }


def socket_route(lay: Layout, pps: int, msgs: list) -> dict:
    """One intra-node step's messages [(x, y, idx)] routed over sockets of
    ``pps`` consecutive ranks (see the module docstring): returns the
    messages of its four parts, {"on", "gather", "cross", "scatter"}."""
    if pps < 1 or lay.ppn % pps:
        raise ValueError("pps must divide ppn")

    def sock(r):
        return r // pps

    on, F, holder, need = [], defaultdict(set), {}, defaultdict(set)
    for x, y, idx in msgs:
        assert lay.node(x) == lay.node(y), "an intra-node step"
        if sock(x) == sock(y):
            on.append((x, y, tuple(idx)))
            continue
        for j in idx:
            F[(sock(x), sock(y))].add(j)
            if holder.setdefault((sock(x), j), x) != x:
                raise AssertionError(f"index {j} held by two ranks of socket {sock(x)}")
            need[(sock(x), sock(y), j)].add(y)

    def order(s, partners):
        return sorted(partners, key=lambda b: (-len(F.get((s, b), ())), b))

    sender, receiver = {}, {}
    sockets = sorted({a for a, _ in F} | {b for _, b in F})
    for s in sockets:
        for k, b in enumerate(order(s, [b for (a, b) in F if a == s])):
            sender[(s, b)] = s * pps + k % pps
        for k, a in enumerate(order(s, [a for (a, b) in F if b == s])):
            receiver[(a, s)] = s * pps + pps - 1 - k % pps
    cross = {(sender[k], receiver[k]): set(v) for k, v in F.items()}
    gather, scatter = defaultdict(set), defaultdict(set)
    for (a, b), idx in F.items():
        q, r = sender[(a, b)], receiver[(a, b)]
        for j in idx:
            h = holder[(a, j)]
            if h != q:
                gather[(h, q)].add(j)
            for y in need[(a, b, j)]:
                if y != r:
                    scatter[(r, y)].add(j)
    return {"on": sorted(on), "gather": _canon(gather), "cross": _canon(cross),
            "scatter": _canon(scatter), "F": {k: sorted(v) for k, v in F.items()},
            "sender": sender, "receiver": receiver}


def socket_plan(csr, lay: Layout, pps: int) -> dict:
    """The NAP plan with a third hierarchy level: sockets of ``pps``
    consecutive ranks route the three intra-node steps (socket_route).  The
    two-level phases stay as they are (they say what each step delivers);
    the socket phases "L0_on", ..., "L2_scatter" say how."""
    out = nap_plan(csr, lay)
    routes = {}
    for ph in ("L0", "L1", "L2"):
        routes[ph] = socket_route(lay, pps, out["phases"][ph])
        for part in SOCKET_PARTS:
            out["phases"][f"{ph}_{part}"] = routes[ph][part]
    out["pps"] = pps
    out["socket_routes"] = routes
    return out


def plan(csr, lay: Layout, mode: str, variant=()) -> dict:
    if mode == "standard":
        return standard_plan(csr, lay)
    if mode == "nap":
        return nap_plan(csr, lay, variant)
    raise ValueError(mode)


def to_arrays(msgs: list):
    """[(src, dst, idx)] -> (src int32, dst int32, ptr int64, idx int32), the
    canonical export format (messages by (src, dst), indices ascending)."""
    src = np.array([m[0] for m in msgs], dtype=np.int32)
    dst = np.array([m[1] for m in msgs], dtype=np.int32)
    ptr = np.zeros(len(msgs) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(m[2]) for m in msgs]) if msgs else []
    idx = np.array([j for m in msgs for j in m[2]], dtype=np.int32)
    return src, dst, ptr, idx
