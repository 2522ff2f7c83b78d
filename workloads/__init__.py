"""Seeded synthetic inputs shaped like the workloads of Bienz, Gropp and Olson,
"Node aware sparse matrix-vector multiplication" (arXiv 1612.08060).

This module only *builds input arrays*: CSR patterns, matrix values, input
vectors, reduced-precision copies of values the caller asks for, and row-block
boundaries given explicitly by a workload.  It holds none of the method's
arithmetic (no partition rule, no communication plan, no product), so that the
CPU oracle and the HIP library can both draw the same inputs from it without
sharing any code that computes a result.

Every generator is deterministic in its arguments: random draws come from
``numpy.random.Generator(PCG64(seed))``.  Grids are numbered
lexicographically (``i = x + nx*y + nx*ny*z``), neighbours outside the domain
are dropped (Dirichlet), and each row stores its columns in ascending order.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CSR", "Workload", "laplacian_2d", "laplacian_3d", "stencil_27", "kkt_like",
    "random_pattern", "vec_uniform", "vec_normal", "to_f32", "bf16_bits",
    "bf16_to_f32", "lognormal_blocks", "config", "digest", "CONFIG_NAMES", "serving_mix",
    "poisson_arrivals",
]


@dataclass
class CSR:
    """A square sparse matrix in CSR form.

    ``rowptr`` is int64 of length ``n + 1``; ``col`` int32 and ``val`` float64
    of length ``nnz``.  Entries of a row are stored in ascending column order
    by every generator here (the library and the oracle accept any order).
    """
    n: int
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def _from_coo(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> CSR:
    """Assemble CSR from COO triples that are already sorted by (row, col)."""
    counts = np.bincount(rows, minlength=n).astype(np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSR(n, rowptr, cols.astype(np.int32), vals.astype(np.float64))


def _stencil(shape, offsets, diag_value: float, off_value: float, n_rows=None) -> CSR:
    """Constant-coefficient stencil on a lexicographic grid.

    ``offsets`` are coordinate offsets (dx, dy, dz).  A neighbour is kept if it
    lies inside the grid and, when ``n_rows`` truncates the grid, below
    ``n_rows``.
    """
    nx, ny, nz = shape
    n = nx * ny * nz if n_rows is None else int(n_rows)
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    # Sort offsets by the linear column shift so each row comes out ascending.
    offs = sorted(offsets, key=lambda o: o[0] + nx * o[1] + nx * ny * o[2])
    rows_l, cols_l, vals_l = [], [], []
    for dx, dy, dz in offs:
        ok = ((x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny)
              & (z + dz >= 0) & (z + dz < nz))
        c = idx + dx + nx * dy + nx * ny * dz
        ok &= (c >= 0) & (c < n)
        r = idx[ok]
        rows_l.append(r)
        cols_l.append(c[ok])
        v = diag_value if (dx, dy, dz) == (0, 0, 0) else off_value
        vals_l.append(np.full(r.size, v, dtype=np.float64))
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l)
    vals = np.concatenate(vals_l)
    # Stable sort by row keeps the ascending-shift order inside each row.
    order = np.argsort(rows, kind="stable")
    return _from_coo(n, rows[order], cols[order], vals[order])


def laplacian_2d(nx: int, ny: int) -> CSR:
    """5-point Poisson stencil, diagonal 4, neighbours -1."""
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0)]
    return _stencil((nx, ny, 1), offs, 4.0, -1.0)


def laplacian_3d(nx: int, ny: int, nz: int) -> CSR:
    """7-point Poisson stencil, diagonal 6, neighbours -1."""
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0),
            (0, 0, -1), (0, 0, 1)]
    return _stencil((nx, ny, nz), offs, 6.0, -1.0)


def stencil_27(n_rows: int, nx: int = 128, ny: int = 128) -> CSR:
    """27-point stencil (diagonal 26, neighbours -1) on an nx x ny x ceil(n/(nx*ny))
    grid truncated to its first ``n_rows`` rows."""
    nz = -(-int(n_rows) // (nx * ny))
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    return _stencil((nx, ny, nz), offs, 26.0, -1.0, n_rows=n_rows)


def kkt_like(n: int, seed: int, band: int = 512, half_lo: int = 10,
             half_hi: int = 20, p_local: float = 0.7) -> CSR:
    """Random symmetric-pattern matrix with a banded plus uniform structure.

    For every row ``i`` a half-degree ``m_i ~ U{half_lo..half_hi}`` is drawn,
    then ``m_i`` columns: with probability ``p_local`` a column
    ``i +- U{1..band}`` (reflected at the ends of ``[0, n)``), otherwise a
    column uniform on ``[0, n)``.  The stored pattern is the union of
    ``(i, j)``, ``(j, i)`` and the diagonal, deduplicated; values are i.i.d.
    N(0, 1) per stored entry.  It stands in for large optimisation (KKT)
    matrices and for the random matrices with a fixed number of nonzeros per
    row used in the paper's experiments.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.integers(half_lo, half_hi + 1, size=n)
    rows = np.repeat(np.arange(n, dtype=np.int64), m)
    k = rows.size
    local = rng.random(k) < p_local
    step = rng.integers(1, band + 1, size=k, dtype=np.int64)
    sign = np.where(rng.random(k) < 0.5, -1, 1)
    j_loc = rows + sign * step
    j_loc = np.where(j_loc < 0, -j_loc, j_loc)
    j_loc = np.where(j_loc >= n, 2 * (n - 1) - j_loc, j_loc)
    j_rnd = rng.integers(0, n, size=k, dtype=np.int64)
    cols = np.where(local, j_loc, j_rnd)
    del local, step, sign, j_loc, j_rnd
    diag = np.arange(n, dtype=np.int64)
    key = np.concatenate([rows * n + cols, cols * n + rows, diag * n + diag])
    del rows, cols
    key = np.unique(key)
    r = key // n
    c = key - r * n
    del key
    vals = rng.standard_normal(r.size)
    return _from_coo(n, r, c, vals)


def random_pattern(n: int, density: float, seed: int, diag: bool = True,
                   empty_rows: int = 0, duplicates: int = 0) -> CSR:
    """Small unstructured (non-symmetric) pattern for brute-force tests.

    ``empty_rows`` rows are emptied, and ``duplicates`` stored entries are
    repeated (a CSR may legally hold a column twice in one row).  Values are
    integers in [-3, 3] so that products are exact in any precision.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    dense = rng.random((n, n)) < density
    if diag:
        np.fill_diagonal(dense, True)
    if empty_rows:
        dense[rng.choice(n, size=min(empty_rows, n), replace=False)] = False
    r, c = np.nonzero(dense)
    if duplicates and r.size:
        pick = rng.choice(r.size, size=duplicates)
        r = np.concatenate([r, r[pick]])
        c = np.concatenate([c, c[pick]])
        order = np.lexsort((c, r))
        r, c = r[order], c[order]
    vals = rng.integers(-3, 4, size=r.size).astype(np.float64)
    return _from_coo(n, r.astype(np.int64), c, vals)


def vec_uniform(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=n)


def vec_normal(n: int, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n)


def to_f32(x: np.ndarray) -> np.ndarray:
    """Round float64 to float32 (round to nearest even)."""
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns (uint16) of ``x``: float64 -> float32 -> bfloat16,
    both steps round to nearest even.  Inputs must be finite."""
    u = to_f32(x).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_to_f32(b: np.ndarray) -> np.ndarray:
    """Widen bfloat16 bit patterns to float32 (exact)."""
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def lognormal_blocks(count: int, seed: int, median: float = 8192.0, sigma: float = 0.6,
                     lo: int = 2048, hi: int = 40960) -> np.ndarray:
    """Block sizes ``clip(round(exp(N(ln median, sigma^2))), lo, hi)``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = np.exp(rng.normal(math.log(median), sigma, size=count))
    return np.clip(np.rint(s), lo, hi).astype(np.int64)


def digest(*arrays: np.ndarray) -> str:
    """SHA-256 over the raw bytes of the given arrays (in order)."""
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


@dataclass
class Workload:
    """A matrix, its process layout and an input vector."""
    name: str
    csr: CSR
    n_p: int
    ppn: int
    v: np.ndarray
    row_starts: np.ndarray | None = None   # explicit block boundaries, or None
    dtypes: tuple = ("f64",)
    meta: dict = field(default_factory=dict)


def serving_mix(count: int = 64, seed: int = 5, n_lo: float = 1e4, n_hi: float = 2e6):
    """Resident matrices of a serving workload.  Matrix k uses generator
    k mod 4 (2D 5-point, 3D 7-point, KKT-like, 3D 27-point) at a size drawn
    log-uniform in [n_lo, n_hi] (snapped to the generator's grid), value type
    floor(k/4) mod 3 (float64, float32, bfloat16), ppn 16 and
    n_p = 16 * max(1, round(N / 32768)).  Returns a list of Workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        target = float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        kind = k % 4
        if kind == 0:
            e = max(16, int(round(target ** 0.5)))
            a = laplacian_2d(e, e)
            name = f"laplace2d_{e}"
        elif kind == 1:
            e = max(8, int(round(target ** (1 / 3))))
            a = laplacian_3d(e, e, e)
            name = f"laplace3d_{e}"
        elif kind == 2:
            n = max(4096, int(target))
            a = kkt_like(n, 1000 + k, band=min(512, n // 8))
            name = f"kkt_like_{n}"
        else:
            n = max(4096, int(target))
            a = stencil_27(n)
            name = f"stencil27_{n}"
        dtype = ("f64", "f32", "bf16")[(k // 4) % 3]
        n_p = 16 * max(1, int(round(a.n / 32768)))
        out.append(Workload(name, a, n_p, 16, vec_uniform(a.n, 2000 + k), dtypes=(dtype,)))
    return out


def poisson_arrivals(n: int, rate_per_s: float, n_mats: int, seed: int):
    """Request trace: (matrix ids uniform over n_mats, arrival times in ns of
    a Poisson process of the given rate)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_per_s, size=n)
    t = np.cumsum(gaps) * 1e9
    ids = rng.integers(0, n_mats, size=n)
    return ids.astype(np.int32), (t - t[0]).astype(np.int64)


CONFIG_NAMES = {
    1: "laplace2d_64x64_np16_ppn4",
    2: "laplace3d_128cube_np1024_ppn16",
    3: "kkt_like_n4194304_np2048_ppn16",
    4: "stencil27_256_lognormal_blocks_ppn16",
}


def config(k: int, scale: int = 0) -> Workload:
    """The paper-shaped workloads.

    1: 2D 5-point Laplacian 64x64, n_p 16, ppn 4, v ~ U(-1,1) (seed 1).
    2: 3D 7-point Laplacian 128^3, n_p 1024, ppn 16, v ~ N(0,1) (seed 2).
    3: KKT-like random matrix, N = 2^22, n_p 2048, ppn 16, values and v N(0,1)
       (seeds 3 and 33); run with float64, float32 and bfloat16 values.
    4: 27-point stencil split into 256 lognormal row blocks (seed 4), ppn 16,
       float32 values, v ~ U(-1,1) (seed 4).

    ``scale`` > 0 shrinks configs 2-4 by 2**scale in rows (same recipe) for
    CPU-sized tests.
    """
    if k == 1:
        a = laplacian_2d(64, 64)
        return Workload(CONFIG_NAMES[1], a, 16, 4, vec_uniform(a.n, 1))
    if k == 2:
        e = 128 >> scale
        a = laplacian_3d(e, e, e)
        n_p = max(16, 1024 >> (3 * scale))
        return Workload(CONFIG_NAMES[2] if scale == 0 else f"laplace3d_{e}cube", a,
                        n_p, 16, vec_normal(a.n, 2))
    if k == 3:
        n = (1 << 22) >> scale
        a = kkt_like(n, 3)
        n_p = max(32, 2048 >> scale)
        return Workload(CONFIG_NAMES[3] if scale == 0 else f"kkt_like_n{n}", a, n_p, 16,
                        vec_normal(n, 33), dtypes=("f64", "f32", "bf16"))
    if k == 4:
        count = max(16, 256 >> scale)
        sizes = lognormal_blocks(count, 4)
        if scale:
            sizes = np.maximum(sizes >> scale, 64)
        row_starts = np.zeros(count + 1, dtype=np.int64)
        np.cumsum(sizes, out=row_starts[1:])
        n = int(row_starts[-1])
        a = stencil_27(n)
        return Workload(CONFIG_NAMES[4] if scale == 0 else f"stencil27_{count}blocks", a,
                        count, 16, vec_uniform(n, 4), row_starts=row_starts,
                        dtypes=("f32",))
    raise ValueError(f"unknown config {k}")
