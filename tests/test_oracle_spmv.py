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


def test_split_order_pins():
    """The split-order product (on-process block, then off-process block, as
    standard_spmv sums it) equals the dense product within rounding, is exact
    on integer inputs, reduces to the plain product for one process, and its
    C and Python evaluations agree bit for bit."""
    from oracle.spmv import spmv_split, spmv_split_rows
    for seed in range(4):
        a = random_pattern(53, 0.12, seed, empty_rows=2, duplicates=4)
        v_int = (np.arange(53) % 5 - 2).astype(np.float64)
        for n_p in (1, 2, 5, 53):
            assert np.array_equal(spmv_split(a, v_int, n_p), brute.matvec(a, v_int))
        a = CSR(a.n, a.rowptr, a.col, np.random.default_rng(seed).standard_normal(a.nnz))
        v = vec_normal(53, seed)
        assert np.array_equal(spmv_split(a, v, 1), spmv.spmv(a, v))
        for n_p in (3, 7):
            w = spmv_split(a, v, n_p, threads=2)
            ref = brute.matvec(a, v)
            assert np.linalg.norm(w - ref) <= 1e-14 * np.linalg.norm(ref)
            assert np.array_equal(spmv_split_rows(a, v, n_p, range(53)), w)
    starts = np.array([0, 4, 5, 30, 53], np.int64)
    w = spmv_split(a, v, 4, row_starts=starts)
    assert np.array_equal(spmv_split_rows(a, v, 4, range(53), row_starts=starts), w)


def test_split_order_differs_from_stored_order():
    """Planted check: a row whose off-process entries come before its
    on-process entry is summed differently by the two routines."""
    from oracle.spmv import spmv_split
    big = 2.0 ** 53
    # 4 rows on 2 processes; row 0 (process 0 owns columns 0, 1) stores
    # (col 2: 1), (col 3: 2^53), (col 0: -2^53)
    a = CSR(4, np.array([0, 3, 4, 5, 6], np.int64), np.array([2, 3, 0, 1, 2, 3], np.int32),
            np.array([1.0, big, -big, 1.0, 1.0, 1.0]))
    v = np.ones(4)
    assert spmv.spmv(a, v)[0] == 0.0          # (1 + 2^53) - 2^53: the 1 is lost
    assert spmv_split(a, v, 2)[0] == 1.0      # (-2^53 + 1) + 2^53: exact


def test_three_way_order_pins():
    """The three-way product (on_process, on_node, off_node blocks in turn, as
    NAPSpMV sums it) is exact on integer inputs, equals the two-way product
    when no block is on-node (one process per node) or none is off-node (one
    node), is within rounding of the dense product otherwise, and its C and
    Python evaluations agree bit for bit."""
    from oracle.spmv import spmv_split, spmv_split3, spmv_split3_rows
    for seed in range(4):
        a = random_pattern(61, 0.12, seed + 10, empty_rows=2, duplicates=4)
        v_int = (np.arange(61) % 7 - 3).astype(np.float64)
        for n_p, ppn in ((1, 1), (4, 2), (6, 3), (61, 61)):
            assert np.array_equal(spmv_split3(a, v_int, n_p, ppn), brute.matvec(a, v_int))
        a = CSR(a.n, a.rowptr, a.col, np.random.default_rng(seed).standard_normal(a.nnz))
        v = vec_normal(61, seed)
        for n_p in (1, 3, 6):
            assert np.array_equal(spmv_split3(a, v, n_p, 1), spmv_split(a, v, n_p))
            assert np.array_equal(spmv_split3(a, v, n_p, n_p), spmv_split(a, v, n_p))
        for n_p, ppn in ((6, 2), (12, 4)):
            w = spmv_split3(a, v, n_p, ppn, threads=2)
            ref = brute.matvec(a, v)
            assert np.linalg.norm(w - ref) <= 1e-14 * np.linalg.norm(ref)
            assert np.array_equal(spmv_split3_rows(a, v, n_p, ppn, range(61)), w)
    starts = np.array([0, 4, 5, 30, 40, 53, 61], np.int64)
    w = spmv_split3(a, v, 6, 3, row_starts=starts)
    assert np.array_equal(spmv_split3_rows(a, v, 6, 3, range(61), row_starts=starts), w)


def test_three_way_order_differs_from_two_way():
    """Planted check: row 0 on process 0 of node 0 (processes 0, 1 on node 0;
    2, 3 on node 1; one row each) stores (col 0: 2^53), (col 2: -2^53),
    (col 1: 1).  Two-way: 2^53, then the off-process entries in stored order,
    -2^53 then 1, gives 1.  Three-way: 2^53, then the on-node 1 (lost to
    rounding), then the off-node -2^53, gives 0."""
    from oracle.spmv import spmv_split, spmv_split3
    big = 2.0 ** 53
    a = CSR(4, np.array([0, 3, 4, 5, 6], np.int64), np.array([0, 2, 1, 1, 2, 3], np.int32),
            np.array([big, -big, 1.0, 1.0, 1.0, 1.0]))
    v = np.ones(4)
    assert spmv_split(a, v, 4)[0] == 1.0
    assert spmv_split3(a, v, 4, 2)[0] == 0.0
    assert spmv_split3(a, v, 4, 1)[0] == 1.0      # no on-node block: two-way order


def test_owner_routine_matches_block_routines():
    """The owner-array routine reproduces the block routines bit for bit on
    contiguous partitions (a second code path), and on a strided partition
    is exact on integer inputs and within rounding of the dense product."""
    from oracle.spmv import owners, spmv_split, spmv_split3, spmv_split_owner
    for seed in range(3):
        a = random_pattern(70, 0.1, seed + 40, empty_rows=2, duplicates=3)
        a = CSR(a.n, a.rowptr, a.col, np.random.default_rng(seed).standard_normal(a.nnz))
        v = vec_normal(70, seed + 3)
        starts = np.array([0, 9, 10, 33, 50, 61, 70], np.int64)
        for n_p, ppn, rs in ((6, 2, None), (6, 3, starts), (7, 7, None), (5, 1, None)):
            own = owners(70, n_p, rs)
            assert np.array_equal(spmv_split_owner(a, v, own, ppn, 2), spmv_split(a, v, n_p, rs))
            assert np.array_equal(spmv_split_owner(a, v, own, ppn, 3),
                                  spmv_split3(a, v, n_p, ppn, rs))
        ref = brute.matvec(a, v)
        for n_p, ppn in ((6, 2), (8, 4)):
            for w in (spmv_split(a, v, n_p, strided=True),
                      spmv_split3(a, v, n_p, ppn, strided=True)):
                assert np.linalg.norm(w - ref) <= 1e-14 * np.linalg.norm(ref)
        ai = CSR(a.n, a.rowptr, a.col, np.round(a.val * 4))
        vi = np.round(v * 4)
        assert np.array_equal(spmv_split3(ai, vi, 8, 4, strided=True), brute.matvec(ai, vi))
    # strided owner: row i on process i mod n_p
    assert owners(10, 4, strided=True).tolist() == [0, 1, 2, 3, 0, 1, 2, 3, 0, 1]


def test_strided_split_order_planted():
    """Row 0 stores (col 1: 1), (col 2: 2^53), (col 4: -2^53), 8 rows on 4
    processes.  Strided (process 0 owns rows and columns 0 and 4): the
    on-process -2^53 first, then 1 and 2^53 in stored order,
    (-2^53 + 1) + 2^53 = 1.  Contiguous (process 0 owns 0 and 1): the
    on-process 1 first, then (1 + 2^53) - 2^53 = 0."""
    from oracle.spmv import spmv_split
    big = 2.0 ** 53
    a = CSR(8, np.array([0, 3, 4, 5, 6, 7, 8, 9, 10], np.int64),
            np.array([1, 2, 4, 1, 2, 3, 4, 5, 6, 7], np.int32),
            np.array([1.0, big, -big, 1, 1, 1, 1, 1, 1, 1]))
    v = np.ones(8)
    assert spmv.spmv(a, v)[0] == 0.0            # (1 + 2^53) - 2^53
    assert spmv_split(a, v, 4, strided=True)[0] == 1.0
    assert spmv_split(a, v, 4)[0] == 0.0        # contiguous: rows 0, 1 own cols 0, 1
