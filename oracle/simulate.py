"""Delivery of vector values along a plan's messages, rank by rank, and the
split local SpMVs, following algorithms standard_spmv (section 2.1) and
local_comm / NAPSpMV (section 4.3).

Test infrastructure (see the package docstring).  Every rank gets its own
host buffers; a "message" is a Python list of values copied from the sender's
buffer; nothing is shared between ranks except what a message carries.  The
simulation asserts that every slot of every ghost list is written exactly
once, with the owner's value, bit for bit.

The split product accumulates, per row, from 0 and in stored order within
each block, first the on-process block and then the off-process block
(standard_spmv, and NAPSpMV under the default two-part reading), or the
on_process, on_node and off_node blocks in that order (NAPSpMV with the
``three_way`` variant): one rounded product and one rounded add per entry.
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np

from .plan_ref import Layout, ghosts


class DeliveryError(AssertionError):
    pass


def _local_v(lay: Layout, v):
    """v|R(r) of every rank, keyed by global index."""
    return [{j: float(v[j]) for j in lay.R(r)} for r in range(lay.n_p)]


def _send(lay, v_loc, r, idx):
    """The pack loop: values of R(r) at global indices idx, read from r's own
    part of v."""
    return [v_loc[r][j] for j in idx]


def _receive(slots, counts, idx, vals, expect=None):
    for j, x in zip(idx, vals):
        if j not in slots:
            continue
        counts[j] += 1
        slots[j] = x


def simulate_standard(csr, lay: Layout, plan: dict, v):
    """standard_spmv on every rank.  Returns (ghost values per rank, w)."""
    gh = ghosts(csr, lay)
    v_loc = _local_v(lay, v)
    inbox = defaultdict(list)
    for phase in ("INTER", "L2"):
        for r, t, idx in plan["phases"][phase]:
            inbox[t].append((idx, _send(lay, v_loc, r, idx)))
    ghost_vals = []
    for t in range(lay.n_p):
        slots = {j: None for j in gh[t]}
        counts = defaultdict(int)
        for idx, vals in inbox[t]:
            for j in idx:
                if j not in slots:
                    raise DeliveryError(f"rank {t} received unneeded index {j}")
            _receive(slots, counts, idx, vals)
        _check(t, gh[t], counts, slots, v)
        ghost_vals.append(slots)
    w = _split_product(csr, lay, v_loc, ghost_vals, three_way=False)
    return ghost_vals, w


def _route_socket(lay: Layout, ph: dict, step: str, held, needs):
    """One intra-node step delivered along its socket routes (phases
    step_on, step_gather, step_cross, step_scatter): on-socket messages go
    directly from the holder's values; holders hand off-socket values to the
    socket sender, which sends them to the socket receiver, which uses the
    ones it needs (``needs(r, j)``) and forwards the others.  ``held[r]`` is
    what rank r holds at the start of the step.  Returns, per rank, j ->
    tuple of the values it received."""
    out = [dict() for _ in range(lay.n_p)]

    def take(r, j, extra=None):
        if j in held[r]:
            return held[r][j]
        if extra is not None and j in extra[r]:
            return extra[r][j]
        raise DeliveryError(f"{step}: rank {r} sends {j} it does not hold")

    for x, y, idx in ph[f"{step}_on"]:
        for j in idx:
            out[y][j] = out[y].get(j, ()) + (take(x, j),)
    sbuf = [dict() for _ in range(lay.n_p)]
    for h, q, idx in ph[f"{step}_gather"]:
        for j in idx:
            sbuf[q][j] = take(h, j)
    rbuf = [dict() for _ in range(lay.n_p)]
    for q, r, idx in ph[f"{step}_cross"]:
        for j in idx:
            if j in rbuf[r]:
                raise DeliveryError(f"{step}: rank {r} received {j} twice off-socket")
            rbuf[r][j] = take(q, j, sbuf)
            if needs(r, j):
                out[r][j] = out[r].get(j, ()) + (rbuf[r][j],)
    for r, y, idx in ph[f"{step}_scatter"]:
        for j in idx:
            if j not in rbuf[r]:
                raise DeliveryError(f"{step}: rank {r} forwards {j} it never received")
            out[y][j] = out[y].get(j, ()) + (rbuf[r][j],)
    return out


def simulate_nap(csr, lay: Layout, plan: dict, v):
    """NAPSpMV on every rank.  Returns (ghost values per rank, w).

    Under the ``dedup`` variant a process also uses, for its own product,
    the values it receives in the on_node -> off_node step.  A plan with a
    socket level (``plan_ref.socket_plan``) delivers the three intra-node
    steps along their socket routes."""
    dedup = "dedup" in plan.get("variant", ())
    gh = ghosts(csr, lay)
    gh_set = [set(g) for g in gh]
    v_loc = _local_v(lay, v)
    ph = plan["phases"]
    sockets = "pps" in plan

    # local_comm(on_node -> on_node): b_{l->l}.
    b_ll = [dict() for _ in range(lay.n_p)]
    if sockets:
        b_ll = _route_socket(lay, ph, "L2", v_loc,
                             lambda r, j: j in gh_set[r] and lay.node(lay.owner(j)) == lay.node(r))
    else:
        for r, t, idx in ph["L2"]:
            assert lay.node(r) == lay.node(t)
            for j, x in zip(idx, _send(lay, v_loc, r, idx)):
                b_ll[t][j] = b_ll[t].get(j, ()) + (x,)
    # local_comm(on_node -> off_node): b_{l->nl}.
    b_lnl = [dict() for _ in range(lay.n_p)]
    if sockets:
        sends = [set() for _ in range(lay.n_p)]
        for s_, q_, idx in ph["INTER"]:
            sends[s_].update(idx)
        got = _route_socket(lay, ph, "L0", v_loc,
                            lambda r, j: j in sends[r] and lay.owner(j) != r)
        for s_ in range(lay.n_p):
            for j, xs in got[s_].items():
                if len(xs) != 1:
                    raise DeliveryError(f"L0: rank {s_} received {j} {len(xs)} times")
                b_lnl[s_][j] = xs[0]
    else:
        for p, s, idx in ph["L0"]:
            assert lay.node(p) == lay.node(s)
            for j, x in zip(idx, _send(lay, v_loc, p, idx)):
                b_lnl[s][j] = x
    # Inter-node pack: own values from v|R, the rest from b_{l->nl}.
    g_recv = [dict() for _ in range(lay.n_p)]
    for s, q, idx in ph["INTER"]:
        assert lay.node(s) != lay.node(q)
        g_send = []
        for j in idx:
            if lay.owner(j) == s:
                g_send.append(v_loc[s][j])
            elif j in b_lnl[s]:
                g_send.append(b_lnl[s][j])
            else:
                raise DeliveryError(f"rank {s} must send {j} but never received it")
        for j, x in zip(idx, g_send):
            if j in g_recv[q]:
                raise DeliveryError(f"rank {q} received {j} twice off-node")
            g_recv[q][j] = x
    # local_comm(off_node -> on_node): forwards from g_recv.
    b_nll = [dict() for _ in range(lay.n_p)]
    if sockets:
        b_nll = _route_socket(lay, ph, "L1", g_recv,
                              lambda r, j: (j in gh_set[r] and j not in g_recv[r]
                                            and lay.node(lay.owner(j)) != lay.node(r)))
    else:
        for q, t, idx in ph["L1"]:
            assert lay.node(q) == lay.node(t)
            for j in idx:
                if j not in g_recv[q]:
                    raise DeliveryError(f"rank {q} forwards {j} it never received")
                b_nll[t][j] = b_nll[t].get(j, ()) + (g_recv[q][j],)

    ghost_vals = []
    for t in range(lay.n_p):
        slots = {j: None for j in gh[t]}
        counts = defaultdict(int)
        for src in (b_ll[t], b_nll[t]):
            for j, xs in src.items():
                if j not in slots:
                    raise DeliveryError(f"rank {t} received unneeded index {j}")
                for x in xs:
                    counts[j] += 1
                    slots[j] = x
        for j, x in g_recv[t].items():       # the receiver's own use
            if j in slots:
                counts[j] += 1
                slots[j] = x
        if dedup:
            for j, x in b_lnl[t].items():    # on-node values received for packing
                if j in slots and lay.node(lay.owner(j)) == lay.node(t):
                    counts[j] += 1
                    slots[j] = x
        _check(t, gh[t], counts, slots, v)
        ghost_vals.append(slots)
    three = "three_way" in plan.get("variant", ())
    w = _split_product(csr, lay, v_loc, ghost_vals, three_way=three)
    return ghost_vals, w


def _check(t, gh_t, counts, slots, v):
    for j in gh_t:
        if counts.get(j, 0) != 1:
            raise DeliveryError(f"rank {t}: ghost {j} written {counts.get(j, 0)} times")
        if np.float64(slots[j]).tobytes() != np.float64(v[j]).tobytes():
            raise DeliveryError(f"rank {t}: ghost {j} holds a wrong value")


def _split_product(csr, lay, v_loc, ghost_vals, three_way: bool):
    """local_spmv on the split blocks of every rank, accumulated into w."""
    w = np.zeros(csr.n)
    for t in range(lay.n_p):
        for i in lay.R(t):
            entries = [(int(csr.col[k]), float(csr.val[k]))
                       for k in range(int(csr.rowptr[i]), int(csr.rowptr[i + 1]))]

            def part(j):
                r = lay.owner(j)
                if r == t:
                    return 0
                return 1 if three_way and lay.node(r) == lay.node(t) else 2

            acc = 0.0
            for block in (0, 1, 2):
                for j, a in entries:
                    if part(j) != block:
                        continue
                    x = v_loc[t][j] if block == 0 else ghost_vals[t][j]
                    acc = acc + a * x
            w[i] = acc
    return w
