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


def ghost_pairs(csr, starts: np.ndarray):
    """All (t, j) with j in gh(t): the sorted, unique off-process columns of
    every rank t (the off_process block of section 2), ordered by (t, j)."""
    n = csr.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(csr.rowptr))
    t = owner(starts, rows)
    del rows
    j = csr.col.astype(np.int64)
    r = owner(starts, j)
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


def standard_plan(csr, n_p: int, ppn: int, given_starts=None) -> dict:
    """D(r, t) for every pair, split into inter-node and intra-node classes."""
    starts = row_starts(csr.n, n_p, given_starts)
    t, j = ghost_pairs(csr, starts)
    r = owner(starts, j)
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


def nap_plan(csr, n_p: int, ppn: int, given_starts=None) -> dict:
    """E(n, m), the T/U mapping, the inter-node messages I and the three
    local steps of section 4, under the readings of ``plan_ref``."""
    starts = row_starts(csr.n, n_p, given_starts)
    n_nodes = n_p // ppn
    t, j = ghost_pairs(csr, starts)
    r = owner(starts, j)
    src_node, dst_node = r // ppn, t // ppn
    offn = src_node != dst_node

    # E(n, m): node-level deduplication of the off-node ghosts.
    nn = np.int64(n_nodes)
    key = np.unique((src_node[offn] * nn + dst_node[offn]) * csr.n + j[offn])
    e_pair, e_j = key // csr.n, key % csr.n
    e_n, e_m = e_pair // nn, e_pair % nn
    pairs, sizes = np.unique(e_pair, return_counts=True)
    p_n, p_m = pairs // nn, pairs % nn

    # T: partners of n by (|E(n, m)| desc, m asc) -> local k mod ppn.
    o = np.lexsort((p_m, -sizes, p_n))
    k = _rank_within(p_n[o])
    t_loc = np.empty(pairs.size, dtype=np.int64)
    t_loc[o] = k % ppn
    # U: senders m of node n by (|E(n, m)| desc, m asc) -> local ppn-1-(k mod ppn).
    vol = {}
    for a, b, s in zip(p_n.tolist(), p_m.tolist(), sizes.tolist()):
        vol[(a, b)] = s
    back = np.array([vol.get((b, a), 0) for a, b in zip(p_n.tolist(), p_m.tolist())],
                    dtype=np.int64)
    o = np.lexsort((p_n, -back, p_m))
    k = _rank_within(p_m[o])
    u_loc = np.empty(pairs.size, dtype=np.int64)
    u_loc[o] = ppn - 1 - (k % ppn)

    send_rank = p_n * ppn + t_loc
    recv_rank = p_m * ppn + u_loc
    pair_of = np.searchsorted(pairs, e_pair)
    i_src, i_dst = send_rank[pair_of], recv_rank[pair_of]

    # on_node -> off_node: owner -> inter-node sender, deduplicated per pair.
    own = owner(starts, e_j)
    need = own != i_src
    l0 = np.unique((own[need] * n_p + i_src[need]) * csr.n + e_j[need])
    l0_src, l0_dst, l0_j = l0 // csr.n // n_p, (l0 // csr.n) % n_p, l0 % csr.n

    # off_node -> on_node: receiver of E(n, m) -> each other user t on m.
    gpair = src_node[offn] * nn + dst_node[offn]
    q = recv_rank[np.searchsorted(pairs, gpair)]
    tt, jj = t[offn], j[offn]
    fwd = q != tt

    # on_node -> on_node: direct, the standard intra-node messages.
    onn = (~offn)
    return {
        "mode": "nap", "starts": starts, "ghost_t": t, "ghost_j": j,
        "pairs": pairs, "pair_sizes": sizes, "send_rank": send_rank,
        "recv_rank": recv_rank, "n_nodes": n_nodes,
        "phases": {
            "INTER": _segments(i_src, i_dst, e_j),
            "L0": _segments(l0_src, l0_dst, l0_j),
            "L1": _segments(q[fwd], tt[fwd], jj[fwd]),
            "L2": _segments(r[onn], t[onn], j[onn]),
        },
    }


def plan(csr, n_p: int, ppn: int, mode: str, given_starts=None) -> dict:
    if mode == "standard":
        return standard_plan(csr, n_p, ppn, given_starts)
    if mode == "nap":
        return nap_plan(csr, n_p, ppn, given_starts)
    raise ValueError(mode)


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
