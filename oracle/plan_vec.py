"""The communication sets of standard SpMV (section 2.1) and NAPSpMV (section 4)
computed with NumPy sorting and uniquing, for matrices too large for the
literal evaluation in ``plan_ref``.

Test infrastructure (see the package docstring).  Every set is formed the
same way as its definition: from the stored entries ``(i, j)`` whose column
lives on another process, grouped and deduplicated with ``numpy.unique`` /
``numpy.lexsort`` (library primitives standing in for set union).  The
readings are those of ``plan_ref`` (module docstring there); this module is
checked against ``plan_ref`` entry by entry on small matrices.

Output format per phase: ``(src int32, dst int32, ptr int64, idx int32)``
with messages sorted by (src, dst) and indices ascending inside a message.
"""
from __future__ import annotations

import numpy as np

PHASES = ("INTER", "L0", "L1", "L2")
VARIANTS = frozenset({"owner_map", "dedup", "split", "three_way"})
SOCKET_PARTS = ("on", "gather", "cross", "scatter")
SOCKET_PHASES = tuple(f"{ph}_{part}" for ph in ("L0", "L1", "L2") for part in SOCKET_PARTS)


def row_starts(n: int, n_p: int, given=None) -> np.ndarray:
    """Block boundaries of the even contiguous partition (section 2); the last
    process takes the N mod n_p remainder rows.  ``given`` overrides."""
    if given is not None:
        s = np.asarray(given, dtype=np.int64)
        if s.size != n_p + 1 or s[0] != 0 or s[-1] != n or np.any(np.diff(s) <= 0):
            raise ValueError("row_starts must rise strictly from 0 to N")
        return s
    b = n // n_p
    s = np.arange(n_p + 1, dtype=np.int64) * b
    s[-1] = n
    return s


def owner(starts: np.ndarray, j: np.ndarray) -> np.ndarray:
    """Rank r with j in R(r)."""
    return np.searchsorted(starts, j, side="right") - 1


def owner_fn(starts, n_p: int):
    """The owner map of a partition: contiguous blocks given by ``starts``,
    or, when ``starts`` is None, the strided partition (row r on process
    r mod n_p, section 5)."""
    if starts is None:
        return lambda j: np.asarray(j, dtype=np.int64) % n_p
    return lambda j: owner(starts, j)


def ghost_pairs(csr, own):
    """All (t, j) with j in gh(t): the sorted, unique off-process columns of
    every rank t (the off_process block of section 2), ordered by (t, j)."""
    n = csr.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(csr.rowptr))
    t = own(rows)
    del rows
    j = csr.col.astype(np.int64)
    r = own(j)
    off = r != t
    key = np.unique(t[off] * n + j[off])
    return key // n, key % n


def _segments(src, dst, idx):
    """Sort triples by (src, dst, idx) and cut them into messages."""
    order = np.lexsort((idx, dst, src))
    src, dst, idx = src[order], dst[order], idx[order]
    if src.size == 0:
        return (np.zeros(0, np.int32), np.zeros(0, np.int32),
                np.zeros(1, np.int64), np.zeros(0, np.int32))
    brk = np.flatnonzero((np.diff(src) != 0) | (np.diff(dst) != 0)) + 1
    heads = np.concatenate([[0], brk])
    ptr = np.concatenate([heads, [src.size]]).astype(np.int64)
    return (src[heads].astype(np.int32), dst[heads].astype(np.int32), ptr,
            idx.astype(np.int32))


def _partition(n, n_p, given_starts, strided):
    if strided:
        if given_starts is not None:
            raise ValueError("a strided partition takes no row_starts")
        if n < n_p:
            raise ValueError("need at least one row per process")
        return None, owner_fn(None, n_p)
    starts = row_starts(n, n_p, given_starts)
    return starts, owner_fn(starts, n_p)


def standard_plan(csr, n_p: int, ppn: int, given_starts=None, strided: bool = False) -> dict:
    """D(r, t) for every pair, split into inter-node and intra-node classes."""
    starts, own = _partition(csr.n, n_p, given_starts, strided)
    t, j = ghost_pairs(csr, own)
    r = own(j)
    inter = (r // ppn) != (t // ppn)
    return {
        "mode": "standard", "starts": starts, "ghost_t": t, "ghost_j": j,
        "phases": {
            "INTER": _segments(r[inter], t[inter], j[inter]),
            "L0": _segments(*(np.zeros(0, np.int64),) * 3),
            "L1": _segments(*(np.zeros(0, np.int64),) * 3),
            "L2": _segments(r[~inter], t[~inter], j[~inter]),
        },
    }


def _rank_within(group: np.ndarray) -> np.ndarray:
    """Position of each element inside its run of equal ``group`` values
    (``group`` already sorted)."""
    k = np.arange(group.size, dtype=np.int64)
    first = np.concatenate([[0], np.flatnonzero(np.diff(group) != 0) + 1]) if group.size else k
    start = np.zeros(group.size, dtype=np.int64)
    start[first] = first
    return k - np.maximum.accumulate(start)


def nap_plan(csr, n_p: int, ppn: int, given_starts=None, variant=(), strided: bool = False) -> dict:
    """E(n, m), the T/U mapping, the inter-node messages I and the three
    local steps of section 4, under the readings and variants of
    ``plan_ref`` (module docstring there)."""
    variant = set(variant)
    if variant - VARIANTS:
        raise ValueError(f"unknown variant(s) {sorted(variant - VARIANTS)}")
    starts, own = _partition(csr.n, n_p, given_starts, strided)
    n_nodes = n_p // ppn
    t, j = ghost_pairs(csr, own)
    r = own(j)
    src_node, dst_node = r // ppn, t // ppn
    offn = src_node != dst_node

    # E(n, m): node-level deduplication of the off-node ghosts.
    nn = np.int64(n_nodes)
    key = np.unique((src_node[offn] * nn + dst_node[offn]) * csr.n + j[offn])
    e_pair, e_j = key // csr.n, key % csr.n
    pairs, sizes = np.unique(e_pair, return_counts=True)
    p_n, p_m = pairs // nn, pairs % nn

    # T: partners of n by (|E(n, m)| desc, m asc) -> local k mod ppn.
    o = np.lexsort((p_m, -sizes, p_n))
    kT = np.empty(pairs.size, dtype=np.int64)
    kT[o] = _rank_within(p_n[o])
    t_loc = kT % ppn
    if "owner_map" in variant:
        # the local process owning the most indices of E(n, m) (lowest on ties)
        pair_of_e = np.searchsorted(pairs, e_pair)
        own_loc = own(e_j) % ppn
        counts = np.zeros((pairs.size, ppn), dtype=np.int64)
        np.add.at(counts, (pair_of_e, own_loc), 1)
        t_loc = counts.argmax(axis=1)
    # U: senders m of node n by (|E(n, m)| desc, m asc) -> local ppn-1-(k mod ppn).
    vol = {}
    for a, b, s in zip(p_n.tolist(), p_m.tolist(), sizes.tolist()):
        vol[(a, b)] = s
    back = np.array([vol.get((b, a), 0) for a, b in zip(p_n.tolist(), p_m.tolist())],
                    dtype=np.int64)
    o = np.lexsort((p_n, -back, p_m))
    kU = np.empty(pairs.size, dtype=np.int64)
    kU[o] = _rank_within(p_m[o])
    u_loc = ppn - 1 - (kU % ppn)

    pair_of = np.searchsorted(pairs, e_pair)
    if "split" in variant:
        # pieces of E(n, m) over several senders/receivers when a node has
        # fewer partners (senders) than processes per node
        n_part = np.bincount(p_n, minlength=n_nodes)[p_n]          # k of the sender node
        n_send = np.bincount(p_m, minlength=n_nodes)[p_m]          # k' of the receiver node
        c_snd = np.where(n_part < ppn, (ppn - kT + n_part - 1) // n_part, 1)
        c_rcv = np.where(n_send < ppn, (ppn - kU + n_send - 1) // n_send, 1)
        e_start = np.searchsorted(e_pair, pairs)                    # first entry of each pair
        pos = np.arange(e_j.size) - e_start[pair_of]                # rank inside E(n, m)
        L = sizes[pair_of]
        c = c_snd[pair_of]
        piece = (pos * c) // L
        # piece containing pos: the largest k with k*L//c <= pos
        piece = np.where(((piece + 1) * L) // c <= pos, piece + 1, piece)
        s_loc = np.where(n_part[pair_of] < ppn, kT[pair_of] + piece * n_part[pair_of], t_loc[pair_of])
        r_idx = piece % c_rcv[pair_of]
        r_loc = np.where(n_send[pair_of] < ppn, ppn - 1 - kU[pair_of] - r_idx * n_send[pair_of],
                         u_loc[pair_of])
        i_src = p_n[pair_of] * ppn + s_loc
        i_dst = p_m[pair_of] * ppn + r_loc
    else:
        send_rank = p_n * ppn + t_loc
        recv_rank = p_m * ppn + u_loc
        i_src, i_dst = send_rank[pair_of], recv_rank[pair_of]

    # on_node -> off_node: owner -> inter-node sender, deduplicated per pair.
    o_e = own(e_j)
    need = o_e != i_src
    l0 = np.unique((o_e[need] * n_p + i_src[need]) * csr.n + e_j[need])
    l0_src, l0_dst, l0_j = l0 // csr.n // n_p, (l0 // csr.n) % n_p, l0 % csr.n

    # off_node -> on_node: receiver of j on the destination node -> each other user.
    recv_key = np.unique((dst_node_of := p_m[pair_of]) * csr.n + e_j)
    recv_sorted = i_dst[np.argsort(dst_node_of * csr.n + e_j, kind="stable")]
    gq = np.searchsorted(recv_key, dst_node[offn] * csr.n + j[offn])
    q = recv_sorted[gq]
    tt, jj = t[offn], j[offn]
    fwd = q != tt

    # on_node -> on_node: direct, the standard intra-node messages.
    onn = ~offn
    l2_src, l2_dst, l2_j = r[onn], t[onn], j[onn]
    if "dedup" in variant:
        drop = np.isin((l2_src * n_p + l2_dst) * csr.n + l2_j,
                       (l0_src * n_p + l0_dst) * csr.n + l0_j)
        l2_src, l2_dst, l2_j = l2_src[~drop], l2_dst[~drop], l2_j[~drop]
    return {
        "mode": "nap", "variant": sorted(variant), "starts": starts, "ghost_t": t,
        "ghost_j": j, "pairs": pairs, "pair_sizes": sizes, "n_nodes": n_nodes,
        "phases": {
            "INTER": _segments(i_src, i_dst, e_j),
            "L0": _segments(l0_src, l0_dst, l0_j),
            "L1": _segments(q[fwd], tt[fwd], jj[fwd]),
            "L2": _segments(l2_src, l2_dst, l2_j),
        },
    }


def plan(csr, n_p: int, ppn: int, mode: str, given_starts=None, variant=(),
         strided: bool = False) -> dict:
    if mode == "standard":
        return standard_plan(csr, n_p, ppn, given_starts, strided)
    if mode == "nap":
        return nap_plan(csr, n_p, ppn, given_starts, variant, strided)
    raise ValueError(mode)


def _select(phase, keep):
    """The messages of a phase for which keep (one bool per message) holds."""
    src, dst, ptr, idx = phase
    k = np.flatnonzero(keep)
    sizes = np.diff(ptr)[k]
    take = np.repeat(ptr[k], sizes) + (np.arange(int(sizes.sum())) -
                                       np.repeat(np.cumsum(sizes) - sizes, sizes))
    return (src[k].astype(np.int32), dst[k].astype(np.int32),
            np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64),
            idx[take.astype(np.int64)].astype(np.int32))


def socket_route(phase, n_p: int, pps: int) -> dict:
    """One intra-node step routed over sockets of ``pps`` consecutive ranks
    (reading in ``plan_ref``'s module docstring): the messages whose ranks
    share a socket stay (``on``); per ordered socket pair (a, b) the union
    F(a, b) of the others' indices goes from one sender of a to one
    receiver of b (``cross``), the holders hand it to the sender first
    (``gather``) and the receiver forwards it (``scatter``)."""
    src, dst, ptr, idx = phase
    sizes = np.diff(ptr)
    x = np.repeat(src.astype(np.int64), sizes)
    y = np.repeat(dst.astype(np.int64), sizes)
    j = idx.astype(np.int64)
    on = _select(phase, src // pps == dst // pps)
    off = (x // pps) != (y // pps)
    x, y, j = x[off], y[off], j[off]
    a, b = x // pps, y // pps
    n_sock = n_p // pps
    big = int(j.max()) + 1 if j.size else 1
    # F(a, b): unique (a, b, j); the holder of (a, j) is unique
    fkey = np.unique((a * n_sock + b) * big + j)
    fab, fj = fkey // big, fkey % big
    fa, fb = fab // n_sock, fab % n_sock
    hkey, hfirst = np.unique(a * big + j, return_index=True)
    hold = x[hfirst]
    if np.unique(a * big + j).size != np.unique((a * big + j) * n_p + x).size:
        raise AssertionError("an index held by two ranks of one socket")
    # socket pairs and their volumes
    pairs, vol = np.unique(fab, return_counts=True)
    pa, pb = pairs // n_sock, pairs % n_sock
    # sender: partners b of a by (|F(a, b)| desc, b asc), k-th -> a*pps + k mod pps
    o = np.lexsort((pb, -vol, pa))
    rank = np.empty(pairs.size, np.int64)
    heads = np.concatenate([[0], np.flatnonzero(np.diff(pa[o]) != 0) + 1])
    run = np.arange(pairs.size) - np.repeat(heads, np.diff(np.concatenate([heads, [pairs.size]])))
    rank[o] = run
    sender = pa * pps + rank % pps
    # receiver: senders a of b by (|F(b, a)| desc, a asc), k-th -> b*pps + pps-1 - k mod pps
    rev = pb * n_sock + pa
    pos = np.searchsorted(pairs, rev)
    back = np.where((pos < pairs.size) & (pairs[np.minimum(pos, pairs.size - 1)] == rev),
                    vol[np.minimum(pos, pairs.size - 1)], 0)
    o = np.lexsort((pa, -back, pb))
    heads = np.concatenate([[0], np.flatnonzero(np.diff(pb[o]) != 0) + 1])
    run = np.arange(pairs.size) - np.repeat(heads, np.diff(np.concatenate([heads, [pairs.size]])))
    rank[o] = run
    receiver = pb * pps + pps - 1 - rank % pps
    # cross: one message per socket pair
    pi = np.searchsorted(pairs, fab)
    cross = _segments(sender[pi], receiver[pi], fj)
    # gather: holder -> sender, unique per pair
    h = hold[np.searchsorted(hkey, fa * big + fj)]
    q = sender[pi]
    g = h != q
    gk = np.unique((h[g] * n_p + q[g]) * big + fj[g])
    gather = _segments(gk // big // n_p, gk // big % n_p, gk % big)
    # scatter: receiver -> every other rank that needs the index
    r = receiver[np.searchsorted(pairs, a * n_sock + b)]
    sc = r != y
    sk = np.unique((r[sc] * n_p + y[sc]) * big + j[sc])
    scatter = _segments(sk // big // n_p, sk // big % n_p, sk % big)
    return {"on": on, "gather": gather, "cross": cross, "scatter": scatter}


def socket_plan(csr, n_p: int, ppn: int, pps: int, given_starts=None,
                strided: bool = False) -> dict:
    """nap_plan plus the socket routes of its three intra-node steps
    (phases "L0_on" ... "L2_scatter")."""
    if pps < 1 or ppn % pps:
        raise ValueError("pps must divide ppn")
    out = nap_plan(csr, n_p, ppn, given_starts, (), strided)
    for ph in ("L0", "L1", "L2"):
        route = socket_route(out["phases"][ph], n_p, pps)
        for part in SOCKET_PARTS:
            out["phases"][f"{ph}_{part}"] = route[part]
    out["pps"] = pps
    return out


def phase_stats(phase, n_p: int) -> dict:
    """Message count, element count, and the per-process maxima the paper
    reports in section 5: most messages and elements sent and received by a
    single process, and the largest single message."""
    src, dst, ptr, _ = phase
    sizes = np.diff(ptr)
    out = {"msgs": int(src.size), "elems": int(sizes.sum())}
    out["max_msgs_sent"] = int(np.bincount(src, minlength=n_p).max()) if src.size else 0
    out["max_elems_sent"] = int(np.bincount(src, weights=sizes, minlength=n_p).max()) if src.size else 0
    out["max_msgs_recv"] = int(np.bincount(dst, minlength=n_p).max()) if src.size else 0
    out["max_elems_recv"] = int(np.bincount(dst, weights=sizes, minlength=n_p).max()) if src.size else 0
    out["max_msg_elems"] = int(sizes.max()) if src.size else 0
    return out


def level_stats(phase, n_p: int, pps: int) -> dict:
    """A third hierarchy level (section 6): the phase's messages split into
    those whose source and destination lie on the same socket of ``pps``
    consecutive ranks, and the others, each with ``phase_stats``."""
    src, dst, ptr, idx = phase
    out = {}
    for side, keep in (("on_socket", src // pps == dst // pps), ("off_socket", src // pps != dst // pps)):
        k = np.flatnonzero(keep)
        sizes = np.diff(ptr)[k]
        sub_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        out[side] = phase_stats((src[k], dst[k], sub_ptr, None), n_p)
    return out
