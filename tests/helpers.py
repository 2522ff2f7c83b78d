"""Shared helpers of the test suite (input assembly only; no method arithmetic)."""
import json
import os

import numpy as np

from workloads import CSR

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def csr_from_rows(rows, vals=None):
    rp = [0]
    col = []
    for r in rows:
        col += list(r)
        rp.append(len(col))
    val = np.ones(len(col)) if vals is None else np.asarray(vals, dtype=np.float64)
    return CSR(len(rows), np.array(rp, np.int64), np.array(col, np.int32), val)


def example_2_1():
    g = load_golden("example_2_1.json")
    return g, csr_from_rows(g["pattern"]["rows"])


def triples(msgs):
    """[(src, dst, idx...)] -> sorted list of (src, dst, tuple(idx))."""
    return sorted((int(s), int(d), tuple(int(j) for j in idx)) for s, d, idx in msgs)


def arrays_to_triples(phase):
    src, dst, ptr, idx = phase
    return [(int(src[k]), int(dst[k]), tuple(int(j) for j in idx[ptr[k]:ptr[k + 1]]))
            for k in range(len(src))]
