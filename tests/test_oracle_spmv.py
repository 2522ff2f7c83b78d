"""The oracle's float64 SpMV against the dense product, exact special cases,
and its row-by-row evaluation."""
import numpy as np

from oracle import brute, spmv
from workloads import CSR, kkt_like, laplacian_2d, laplacian_3d, random_pattern, vec_normal


def test_dense_bruteforce():
    for seed in range(6):
        a = random_pattern(37, 0.15, seed, empty_rows=2, duplicates=5)
        a = CSR(a.n, a.rowptr, a.col, np.random.default_rng(seed).standard_normal(a.nnz))
        v = vec_normal(37, seed)
        w = spmv.spmv(a, v)
        ref = brute.matvec(a, v)
        assert np.linalg.norm(w - ref) <= 1e-14 * np.linalg.norm(ref)


def test_integer_inputs_exact():
    a = random_pattern(60, 0.2, 9, duplicates=7)
    v = (np.arange(60) % 7 - 3).astype(np.float64)
    assert np.array_equal(spmv.spmv(a, v), brute.matvec(a, v))


def _boundary_count(coords, dims):
    return sum((c == 0) + (c == d - 1) for c, d in zip(coords, dims))


def test_laplacian_times_constant():
    """A 1 is zero on interior rows and counts missing neighbours on the
    boundary (4 - #neighbours in 2D, 6 - #neighbours in 3D)."""
    a = laplacian_2d(64, 64)
    w = spmv.spmv(a, np.ones(a.n))
    x, y = np.arange(a.n) % 64, np.arange(a.n) // 64
    expect = np.array([_boundary_count((xx, yy), (64, 64)) for xx, yy in zip(x, y)], float)
    assert np.array_equal(w, expect)
    b = laplacian_3d(16, 12, 10)
    w = spmv.spmv(b, np.ones(b.n))
    i = np.arange(b.n)
    expect = np.array([_boundary_count((k % 16, (k // 16) % 12, k // 192), (16, 12, 10))
                       for k in i], float)
    assert np.array_equal(w, expect)


def test_rows_match_full_product_bitwise():
    a = kkt_like(1 << 12, 5)
    v = vec_normal(a.n, 6)
    w = spmv.spmv(a, v, threads=3)
    rows = [0, 1, 17, 2048, a.n - 1]
    assert np.array_equal(spmv.spmv_rows(a, v, rows), w[rows])
    assert np.array_equal(spmv.spmv(a, v, threads=1), w)


def test_empty_matrix_rows():
    a = CSR(4, np.array([0, 0, 0, 0, 0], np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert np.array_equal(spmv.spmv(a, np.ones(4)), np.zeros(4))
