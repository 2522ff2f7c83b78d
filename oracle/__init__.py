"""CPU oracle for node-aware parallel SpMV (Bienz, Gropp, Olson, arXiv 1612.08060).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only the test suite, the smoke check of
the entry module and the CPU-baseline leg of the benchmark use it.  It shares
no code with the HIP library (no kernels, headers, helpers or tables); both
sides only draw their inputs from the ``workloads`` module, which holds none
of the method's arithmetic.

Contents
--------
plan_ref   literal, set-based evaluation of every communication set of the
           paper (standard SpMV of section 2.1 and NAPSpMV of section 4),
           one stored entry at a time.  For tiny and small matrices.
plan_vec   the same sets with NumPy sorting and uniquing, for large matrices;
           cross-checked against plan_ref on small ones.
brute      definitions evaluated quantifier by quantifier over a dense
           pattern (tiny matrices only), and the dense matrix-vector product.
simulate   moves every vector value along its message path, as algorithms
           standard_spmv and NAPSpMV do, into per-process host buffers; checks
           that each ghost slot is written exactly once and runs the split
           local SpMVs.
spmv       plain float64 CSR SpMV (the definition w = A v) in C, plus a
           row-by-row Python evaluation for sampled rows.

Pins (tests marked "not gpu") tie each part to something other than itself:
the worked example of section 2 (every printed table, with the errata noted
in the golden file), hand-derived closed forms for the 2D and 3D Laplacian
layouts, special cases (ppn = 1, ppn = n_p, n_p = 1), invariants the paper
states, and brute force on tiny inputs.

Parity unpinned: the assignment of partner nodes to local processes when a
node has more partners than processes per node (the paper is silent) is
pinned only by invariants (every partner assigned exactly once, per-process
partner counts differ by at most one), not by a value the paper prints.
"""
