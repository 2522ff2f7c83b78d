"""Brute force over a dense pattern, for tiny matrices only.

Test infrastructure (see the package docstring).  Each communication set is
evaluated straight from its quantifiers ("there exist i in R(t) and j in R(r)
with A_ij != 0"), by looping over ranks, nodes and dense row/column ranges.
This is a different route from ``plan_ref`` (which walks the stored entries
once) and is used to pin it.  The product is the dense matrix times the
vector with NumPy (a library matmul), which pins the CSR SpMV of ``spmv``.
"""
from __future__ import annotations

import numpy as np


def dense(csr) -> np.ndarray:
    """Dense float64 matrix; duplicate stored entries are summed."""
    a = np.zeros((csr.n, csr.n))
    for i in range(csr.n):
        for k in range(int(csr.rowptr[i]), int(csr.rowptr[i + 1])):
            a[i, csr.col[k]] += csr.val[k]
    return a


def pattern(csr) -> np.ndarray:
    """Structural pattern: True where an entry is stored (even a stored zero)."""
    s = np.zeros((csr.n, csr.n), dtype=bool)
    for i in range(csr.n):
        s[i, csr.col[csr.rowptr[i]:csr.rowptr[i + 1]]] = True
    return s


def matvec(csr, v: np.ndarray) -> np.ndarray:
    return dense(csr) @ np.asarray(v, dtype=np.float64)


def blocks(n: int, n_p: int, row_starts=None, strided: bool = False):
    """R(r) as Python ranges, with the remainder rows on the last rank; or,
    strided, rows r, r + n_p, r + 2 n_p, ..."""
    if strided:
        return [range(r, n, n_p) for r in range(n_p)]
    if row_starts is None:
        b = n // n_p
        row_starts = [b * r for r in range(n_p)] + [n]
    return [range(int(row_starts[r]), int(row_starts[r + 1])) for r in range(n_p)]


def _exists(S, rows, cols) -> bool:
    return any(S[i, j] for i in rows for j in cols)


def standard_sets(csr, n_p: int, ppn: int, row_starts=None, strided: bool = False) -> dict:
    """P(r) and D(r, t), straight from their quantifiers."""
    S = pattern(csr)
    R = blocks(csr.n, n_p, row_starts, strided)
    P = {r: [t for t in range(n_p) if t != r and _exists(S, R[t], R[r])] for r in range(n_p)}
    D = {}
    for r in range(n_p):
        for t in P[r]:
            D[(r, t)] = [j for j in R[r] if any(S[i, j] for i in R[t])]
    return {"P": P, "D": D}


def node_sets(csr, n_p: int, ppn: int, row_starts=None, strided: bool = False):
    """N(n) and E(n, m), straight from their quantifiers over (p, q)."""
    S = pattern(csr)
    R = blocks(csr.n, n_p, row_starts, strided)
    nodes = n_p // ppn
    rank = lambda p, n: n * ppn + p  # noqa: E731
    E = {}
    for n in range(nodes):
        for m in range(nodes):
            if m == n:
                continue
            idx = [j for p in range(ppn) for j in R[rank(p, n)]
                   if any(S[i, j] for q in range(ppn) for i in R[rank(q, m)])]
            if idx:
                E[(n, m)] = sorted(idx)
    N = {n: sorted(m for (a, m) in E if a == n) for n in range(nodes)}
    return N, E


def mapping(n_p: int, ppn: int, E: dict):
    """The T/U assignment, from a dense node-to-node volume matrix and
    ``numpy.lexsort`` (a second route to the rule of ``plan_ref.mapping``)."""
    nodes = n_p // ppn
    vol = np.zeros((nodes, nodes), dtype=np.int64)
    for (n, m), idx in E.items():
        vol[n, m] = len(idx)
    send_rank, recv_rank = {}, {}
    for n in range(nodes):
        partners = np.flatnonzero(vol[n] > 0)
        order = partners[np.lexsort((partners, -vol[n, partners]))]
        for k, m in enumerate(order):
            send_rank[(n, int(m))] = n * ppn + k % ppn
        senders = np.flatnonzero(vol[:, n] > 0)
        order = senders[np.lexsort((senders, -vol[n, senders]))]
        for k, m in enumerate(order):
            recv_rank[(int(m), n)] = n * ppn + ppn - 1 - k % ppn
    return send_rank, recv_rank


def nap_sets(csr, n_p: int, ppn: int, row_starts=None, strided: bool = False) -> dict:
    """I, and J of the three local steps, from their quantifiers, given E and
    the mapping."""
    S = pattern(csr)
    R = blocks(csr.n, n_p, row_starts, strided)
    N, E = node_sets(csr, n_p, ppn, row_starts, strided)
    send_rank, recv_rank = mapping(n_p, ppn, E)
    node = lambda r: r // ppn  # noqa: E731
    I = {(send_rank[k], recv_rank[k]): E[k] for k in E}
    J0, J1, J2 = {}, {}, {}
    for p in range(n_p):
        for s in range(n_p):
            if s == p or node(s) != node(p):
                continue
            # J0: values of R(p) that s sends off-node.
            out = [j for j in R[p] if any(j in idx for (a, b), idx in I.items() if a == s)]
            if out:
                J0[(p, s)] = out
            # J1: values p received off-node that a row of s uses.
            got = sorted({j for (a, b), idx in I.items() if b == p for j in idx})
            fw = [j for j in got if any(S[i, j] for i in R[s])]
            if fw:
                J1[(p, s)] = fw
            # J2: values of R(p) that a row of s uses.
            loc = [j for j in R[p] if any(S[i, j] for i in R[s])]
            if loc:
                J2[(p, s)] = loc
    return {"N": N, "E": E, "send_rank": send_rank, "recv_rank": recv_rank,
            "I": I, "J0": J0, "J1": J1, "J2": J2}


def socket_sets(csr, n_p: int, ppn: int, pps: int, row_starts=None) -> dict:
    """The socket routes of the three intra-node steps (reading in
    ``plan_ref``), each set straight from its quantifier over the steps' J
    sets of ``nap_sets``, the mapping from a dense socket-to-socket volume
    matrix and ``numpy.lexsort``.  Returns {step: {part: {(src, dst):
    sorted list}}} for step in J0, J1, J2 and part in on, gather, cross,
    scatter."""
    b = nap_sets(csr, n_p, ppn, row_starts)
    n_sock = n_p // pps
    per_node = ppn // pps
    sock = lambda r: r // pps  # noqa: E731
    out = {}
    for key in ("J0", "J1", "J2"):
        J = b[key]
        on = {k: v for k, v in J.items() if sock(k[0]) == sock(k[1])}
        F = {}
        for s in range(n_sock):
            for s2 in range(n_sock):
                if s2 == s or s // per_node != s2 // per_node:
                    continue
                idx = sorted({j for (x, y), v in J.items() if sock(x) == s and sock(y) == s2
                              for j in v})
                if idx:
                    F[(s, s2)] = idx
        vol = np.zeros((n_sock, n_sock), dtype=np.int64)
        for (s, s2), idx in F.items():
            vol[s, s2] = len(idx)
        send, recv = {}, {}
        for s in range(n_sock):
            partners = np.flatnonzero(vol[s] > 0)
            for k, s2 in enumerate(partners[np.lexsort((partners, -vol[s, partners]))]):
                send[(s, int(s2))] = s * pps + k % pps
            senders = np.flatnonzero(vol[:, s] > 0)
            for k, s2 in enumerate(senders[np.lexsort((senders, -vol[s, senders]))]):
                recv[(int(s2), s)] = s * pps + pps - 1 - k % pps
        cross = {(send[k], recv[k]): v for k, v in F.items()}
        gather, scatter = {}, {}
        for h in range(n_p):
            for q in range(sock(h) * pps, (sock(h) + 1) * pps):
                if q == h:
                    continue
                # indices h holds for another socket whose sender is q
                idx = sorted({j for (s, s2), v in F.items() if send[(s, s2)] == q
                              for j in v
                              if any(j in J.get((h, y), ()) for y in range(s2 * pps, (s2 + 1) * pps))})
                if idx:
                    gather[(h, q)] = idx
        for y in range(n_p):
            for r in range(sock(y) * pps, (sock(y) + 1) * pps):
                if r == y:
                    continue
                # indices y needs from another socket whose receiver is r
                idx = sorted({j for (s, s2), v in F.items() if recv[(s, s2)] == r
                              for j in v
                              if any(j in J.get((x, y), ()) for x in range(s * pps, (s + 1) * pps))})
                if idx:
                    scatter[(r, y)] = idx
        out[key] = {"on": on, "gather": gather, "cross": cross, "scatter": scatter}
    return out
