"""Seeded synthetic CSR inputs shaped like the paper's workloads.

This module produces input matrices only.  It holds no part of the product
C = A*B: no multiplication, merge, count or sum of the method is computed
here, so that both the CPU oracle and the GPU library can consume the same
inputs without sharing any of the method's arithmetic.

Every generator returns a :class:`CSR` whose rows have strictly increasing
column indices (the storage format of Section II-A.3 of the paper), int32
column indices, float64 values and an int32 row-pointer array whenever the
number of stored entries fits in int32 (int64 otherwise).

Random streams come from numpy's PCG64 bit generator seeded with the caller's
seed, so every input is reproducible from ``(generator, parameters, seed)``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR",
    "from_dense",
    "identity",
    "permutation",
    "laplacian_2d_5pt",
    "tridiag_kron2",
    "stencil_3d_27pt",
    "erdos_renyi_rows",
    "rmat",
    "aggregation_p",
    "aggregation_pt",
    "amg_batch",
    "random_csr",
    "csr_transpose",
    "row_block",
]

_I32_MAX = np.iinfo(np.int32).max


@dataclass
class CSR:
    """A CSR matrix held in host memory (numpy arrays)."""

    rows: int
    cols: int
    rpt: np.ndarray  # int32 or int64, rows + 1 entries, rpt[0] == 0
    col: np.ndarray  # int32, strictly increasing within each row
    val: np.ndarray  # float64

    @property
    def nnz(self) -> int:
        return int(self.rpt[-1]) if self.rows > 0 else 0

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rpt.astype(np.int64))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.rows, self.cols), dtype=np.float64)
        r = np.repeat(np.arange(self.rows), self.row_lengths())
        d[r, self.col.astype(np.int64)] = self.val
        return d


def _rpt_from_lengths(lengths: np.ndarray) -> np.ndarray:
    lengths = np.asarray(lengths, dtype=np.int64)
    rpt = np.zeros(lengths.size + 1, dtype=np.int64)
    np.cumsum(lengths, out=rpt[1:])
    if rpt[-1] <= _I32_MAX:
        return rpt.astype(np.int32)
    return rpt


def _from_sorted_coo(rows: int, cols: int, r: np.ndarray, c: np.ndarray, v: np.ndarray) -> CSR:
    lengths = np.bincount(r, minlength=rows) if r.size else np.zeros(rows, dtype=np.int64)
    return CSR(rows, cols, _rpt_from_lengths(lengths), c.astype(np.int32), v.astype(np.float64))


def from_dense(d: np.ndarray, pattern: np.ndarray | None = None) -> CSR:
    """CSR of a dense array.  ``pattern`` (bool) selects the stored entries;
    by default every nonzero is stored.  Stored zeros are allowed."""
    d = np.asarray(d, dtype=np.float64)
    if pattern is None:
        pattern = d != 0
    r, c = np.nonzero(pattern)
    return _from_sorted_coo(d.shape[0], d.shape[1], r, c, d[r, c])


def identity(n: int, scale: float = 1.0) -> CSR:
    idx = np.arange(n)
    return _from_sorted_coo(n, n, idx, idx, np.full(n, scale))


def permutation(perm: np.ndarray) -> CSR:
    """The matrix with a single 1 at (i, perm[i]) in every row."""
    perm = np.asarray(perm)
    n = perm.size
    return _from_sorted_coo(n, n, np.arange(n), perm, np.ones(n))


def laplacian_2d_5pt(n: int, center: float = 4.0, off: float = -1.0) -> CSR:
    """5-point Laplacian on an n x n grid, point (x, y) -> row x + n*y."""
    x, y = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ids = (x + n * y).ravel()
    xs, ys = x.ravel(), y.ravel()
    # neighbour offsets in increasing column order: -n, -1, 0, +1, +n
    offs = [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]
    masks, cols, vals = [], [], []
    for dx, dy in offs:
        m = (xs + dx >= 0) & (xs + dx < n) & (ys + dy >= 0) & (ys + dy < n)
        masks.append(m)
        cols.append(ids + dx + n * dy)
        vals.append(np.full(ids.size, center if (dx, dy) == (0, 0) else off))
    return _stack_offsets(n * n, n * n, ids, masks, cols, vals)


def _stack_offsets(rows, ncols, ids, masks, cols, vals) -> CSR:
    """Assemble CSR from per-offset candidate entries whose columns already
    increase with the offset index for every row."""
    m = np.stack(masks)  # (noff, rows)
    c = np.stack(cols)
    v = np.stack(vals)
    order = np.argsort(ids, kind="stable")
    m, c, v = m[:, order], c[:, order], v[:, order]
    # row-major traversal: for each row, the valid offsets in offset order
    mt, ct, vt = m.T, c.T, v.T
    lengths = mt.sum(axis=1)
    return CSR(rows, ncols, _rpt_from_lengths(lengths), ct[mt].astype(np.int32), vt[mt].astype(np.float64))


def tridiag_kron2(n: int) -> CSR:
    """S (x) S for the 1-D all-ones tridiagonal S: the all-ones 9-point stencil
    on an n x n grid (row x + n*y)."""
    x, y = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    ids = (x + n * y).ravel()
    xs, ys = x.ravel(), y.ravel()
    masks, cols, vals = [], [], []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            m = (xs + dx >= 0) & (xs + dx < n) & (ys + dy >= 0) & (ys + dy < n)
            masks.append(m)
            cols.append(ids + dx + n * dy)
            vals.append(np.ones(ids.size))
    return _stack_offsets(n * n, n * n, ids, masks, cols, vals)


def stencil_3d_27pt(n: int, center: float = 26.0, off: float = -1.0) -> CSR:
    """27-point stencil on an n^3 cube, point (x, y, z) -> x + n*(y + n*z)."""
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    xs, ys, zs = x.ravel(), y.ravel(), z.ravel()
    ids = xs + n * (ys + n * zs)
    masks, cols, vals = [], [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                m = ((xs + dx >= 0) & (xs + dx < n) & (ys + dy >= 0) & (ys + dy < n)
                     & (zs + dz >= 0) & (zs + dz < n))
                masks.append(m)
                cols.append(ids + dx + n * (dy + n * dz))
                vals.append(np.full(ids.size, center if (dx, dy, dz) == (0, 0, 0) else off))
    return _stack_offsets(n ** 3, n ** 3, ids, masks, cols, vals)


def erdos_renyi_rows(n: int, k: int, seed: int, lo: float = -1.0, hi: float = 1.0,
                     ncols: int | None = None) -> CSR:
    """n x ncols matrix with exactly k distinct uniformly drawn columns per row
    (rows with a repeated column are redrawn whole), values U[lo, hi) drawn
    after the pattern, in row-major order."""
    ncols = n if ncols is None else ncols
    if k > ncols:
        raise ValueError("k exceeds the number of columns")
    rng = np.random.Generator(np.random.PCG64(seed))
    c = rng.integers(0, ncols, size=(n, k), dtype=np.int64)
    c.sort(axis=1)
    while True:
        bad = np.nonzero((c[:, 1:] == c[:, :-1]).any(axis=1))[0] if k > 1 else np.zeros(0, np.int64)
        if bad.size == 0:
            break
        redraw = rng.integers(0, ncols, size=(bad.size, k), dtype=np.int64)
        redraw.sort(axis=1)
        c[bad] = redraw
    val = rng.uniform(lo, hi, size=n * k)
    return CSR(n, ncols, _rpt_from_lengths(np.full(n, k)), c.ravel().astype(np.int32), val)


def rmat(scale: int, edge_factor: int, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, lo: float = 0.0, hi: float = 1.0) -> CSR:
    """Directed R-MAT graph (recursive quadrant choice with probabilities
    a, b, c, d = 1-a-b-c at every level, no noise, no permutation), self loops
    kept, duplicate edges removed, values U[lo, hi) drawn after deduplication
    in sorted (row, col) order."""
    n = 1 << scale
    m = edge_factor * n
    rng = np.random.Generator(np.random.PCG64(seed))
    r = np.zeros(m, dtype=np.int64)
    q = np.zeros(m, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for level in range(scale):
        u = rng.random(m)
        bit = np.int64(1) << np.int64(scale - 1 - level)
        row_bit = u >= ab                      # quadrants c, d
        col_bit = ((u >= a) & (u < ab)) | (u >= abc)  # quadrants b, d
        r += row_bit * bit
        q += col_bit * bit
        del u, row_bit, col_bit
    key = np.unique((r << np.int64(scale)) | q)
    del r, q
    rows = key >> np.int64(scale)
    cols = key & np.int64(n - 1)
    val = rng.uniform(lo, hi, size=key.size)
    return _from_sorted_coo(n, n, rows, cols, val)


def _agg_index(n: int):
    m = (n + 1) // 2
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    fine = (x + n * (y + n * z)).ravel()
    coarse = ((x // 2) + m * ((y // 2) + m * (z // 2))).ravel()
    return m, fine, coarse


def aggregation_p(n: int) -> CSR:
    """Piecewise-constant prolongation over 2x2x2 aggregates of an n^3 grid:
    P[fine, agg(fine)] = 1, with agg taking x//2, y//2, z//2 per axis."""
    m, fine, coarse = _agg_index(n)
    order = np.argsort(fine)
    return _from_sorted_coo(n ** 3, m ** 3, fine[order], coarse[order], np.ones(fine.size))


def aggregation_pt(n: int) -> CSR:
    """The transpose of :func:`aggregation_p`, built directly: row J lists the
    fine points of aggregate J in increasing order."""
    m, fine, coarse = _agg_index(n)
    order = np.lexsort((fine, coarse))
    return _from_sorted_coo(m ** 3, n ** 3, coarse[order], fine[order], np.ones(fine.size))


def amg_batch(count: int, seed: int, edge_lo: int = 16, edge_hi: int = 64):
    """``count`` Galerkin problems: for each, a cube edge n ~ U{edge_lo..edge_hi},
    the 27-point stencil A (26 / -1), the aggregation P and its transpose."""
    rng = np.random.Generator(np.random.PCG64(seed))
    edges = rng.integers(edge_lo, edge_hi + 1, size=count)
    out = []
    for n in edges:
        n = int(n)
        out.append((n, stencil_3d_27pt(n), aggregation_p(n), aggregation_pt(n)))
    return out


def amg_levels(n: int, coarsest: int = 2):
    """The grid edges of an aggregation hierarchy on an n^3 cube: n, ceil(n/2),
    ... down to the first edge <= ``coarsest``, with the prolongation and its
    transpose of every level but the last: [(edge, P, Pt), ...]."""
    out = []
    while n > coarsest:
        out.append((n, aggregation_p(n), aggregation_pt(n)))
        n = (n + 1) // 2
    return out


def random_csr(rows: int, cols: int, density: float, seed: int, integer_values: bool = False,
               empty_row_frac: float = 0.0, lo: float = -1.0, hi: float = 1.0) -> CSR:
    """Bernoulli(density) pattern; values U[lo, hi) or small nonzero integers in
    [-4, 4].  A fraction of rows can be forced empty."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pat = rng.random((rows, cols)) < density
    if empty_row_frac > 0 and rows > 0:
        pat[rng.random(rows) < empty_row_frac] = False
    if integer_values:
        v = rng.integers(1, 5, size=(rows, cols)).astype(np.float64)
        v *= np.where(rng.random((rows, cols)) < 0.5, -1.0, 1.0)
    else:
        v = rng.uniform(lo, hi, size=(rows, cols))
    return from_dense(np.where(pat, v, 0.0), pattern=pat)


def csr_transpose(A: CSR) -> CSR:
    """Index reshuffle to the transpose (stable, so columns stay sorted)."""
    r = np.repeat(np.arange(A.rows, dtype=np.int64), A.row_lengths())
    c = A.col.astype(np.int64)
    order = np.lexsort((r, c))
    return _from_sorted_coo(A.cols, A.rows, c[order], r[order], A.val[order])


def row_block(A: CSR, begin: int, end: int) -> CSR:
    """Rows [begin, end) of A as a CSR of their own (same column count)."""
    lo, hi = int(A.rpt[begin]), int(A.rpt[end])
    rpt = A.rpt[begin:end + 1].astype(np.int64) - lo
    return CSR(end - begin, A.cols, _rpt_from_lengths(np.diff(rpt)), A.col[lo:hi].copy(), A.val[lo:hi].copy())
