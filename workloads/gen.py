"""Seeded generators for the sparse matrices that drive PB-SpGEMM.

Every generator is deterministic in its seed (numpy PCG64 via
``default_rng``).  Shapes and distributions follow the paper's workloads:

* Erdos-Renyi (ER): a matrix with d nonzeros per column placed uniformly at
  random (Section 2.1, "Notations").  Here each column gets exactly d
  *distinct* rows, as that definition reads.
* R-MAT / Graph500 (Section 4.3, "Dataset"): recursive quadrant choice with
  (a, b, c, d) = (0.57, 0.19, 0.19, 0.05), symmetrised, duplicates removed.
* Batched uneven ER products and an AMG Galerkin triple product are
  workload shapes beyond the paper (see the design notes); they only use the
  same ER building block or a closed-form stencil construction.

Matrices are held in :class:`Csx`: ``ptr`` int64, ``idx`` int32 (strictly
increasing inside each column / row), ``val`` float64.  ``fmt`` says whether
``ptr`` indexes columns (``"csc"``) or rows (``"csr"``).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Csx",
    "csc_to_csr",
    "csr_to_csc",
    "er_csc",
    "er_problem",
    "identity",
    "random_sparse",
    "rmat_symmetric",
    "batched_er_sizes",
    "batched_er_problems",
    "amg_problem",
]


@dataclasses.dataclass
class Csx:
    """A compressed sparse matrix (CSC or CSR) with int64 pointers."""

    nrows: int
    ncols: int
    ptr: np.ndarray  # int64, (ncols+1) for CSC, (nrows+1) for CSR
    idx: np.ndarray  # int32 minor indices, strictly increasing per major slice
    val: np.ndarray  # float64
    fmt: str  # "csc" or "csr"

    @property
    def nnz(self) -> int:
        return int(self.ptr[-1])

    @property
    def nmajor(self) -> int:
        return self.ncols if self.fmt == "csc" else self.nrows

    @property
    def nminor(self) -> int:
        return self.nrows if self.fmt == "csc" else self.ncols

    def major_counts(self) -> np.ndarray:
        return np.diff(self.ptr)

    def transpose_view(self) -> "Csx":
        """The same arrays read as the transpose in the other format.

        CSC arrays of A are the CSR arrays of A^T and vice versa; no data moves.
        """
        other = "csr" if self.fmt == "csc" else "csc"
        return Csx(self.ncols, self.nrows, self.ptr, self.idx, self.val, other)

    def check(self) -> None:
        """Structural validity: monotone pointers, sorted distinct indices."""
        assert self.fmt in ("csc", "csr")
        assert self.ptr.dtype == np.int64 and self.idx.dtype == np.int32
        assert self.val.dtype in (np.float64,)
        assert self.ptr.shape == (self.nmajor + 1,)
        assert self.ptr[0] == 0 and np.all(np.diff(self.ptr) >= 0)
        assert self.idx.shape == (self.nnz,) and self.val.shape == (self.nnz,)
        if self.nnz:
            assert self.idx.min() >= 0 and self.idx.max() < self.nminor
            d = np.diff(self.idx.astype(np.int64))
            starts = self.ptr[1:-1]
            inside = np.ones(self.nnz - 1, dtype=bool) if self.nnz > 1 else np.zeros(0, bool)
            # positions p where p and p+1 are in different slices are exempt
            cut = starts[(starts > 0) & (starts < self.nnz)] - 1
            inside[cut] = False
            assert np.all(d[inside] > 0), "indices must strictly increase in a slice"


def _compress(nmajor: int, major: np.ndarray, minor: np.ndarray, val: np.ndarray):
    """Group COO entries by major index, keeping the incoming order inside a
    group (stable counting sort).  Returns ptr, idx, val."""
    major = np.asarray(major, dtype=np.int64)
    order = np.argsort(major, kind="stable")
    counts = np.bincount(major, minlength=nmajor).astype(np.int64)
    ptr = np.zeros(nmajor + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return ptr, np.ascontiguousarray(minor[order], dtype=np.int32), np.ascontiguousarray(
        val[order], dtype=np.float64
    )


def _expand_major(ptr: np.ndarray) -> np.ndarray:
    return np.repeat(np.arange(len(ptr) - 1, dtype=np.int64), np.diff(ptr))


def csc_to_csr(a: Csx) -> Csx:
    """Same matrix, CSR storage (stable transpose of the storage order)."""
    assert a.fmt == "csc"
    cols = _expand_major(a.ptr)
    ptr, idx, val = _compress(a.nrows, a.idx, cols, a.val)
    return Csx(a.nrows, a.ncols, ptr, idx, val, "csr")


def csr_to_csc(b: Csx) -> Csx:
    """Same matrix, CSC storage."""
    assert b.fmt == "csr"
    rows = _expand_major(b.ptr)
    ptr, idx, val = _compress(b.ncols, b.idx, rows, b.val)
    return Csx(b.nrows, b.ncols, ptr, idx, val, "csc")


def _values(rng: np.random.Generator, nnz: int, kind: str) -> np.ndarray:
    if kind == "uniform":  # U[0,1)
        return rng.random(nnz)
    if kind == "signed":  # U[-1,1)
        return 2.0 * rng.random(nnz) - 1.0
    if kind == "int":  # small nonzero integers: every sum of products is exact
        v = rng.integers(-3, 4, size=nnz).astype(np.float64)
        v[v == 0] = 1.0
        return v
    if kind == "ones":
        return np.ones(nnz)
    raise ValueError(kind)


def er_csc(n: int, d: int, seed: int, nrows: int | None = None, values: str = "uniform") -> Csx:
    """ER matrix with exactly ``d`` distinct uniformly random rows per column.

    Draw order: an (ncols, d) block of rows; columns holding a repeated row are
    redrawn whole (in column order) until every column is distinct; then the
    values.  Rows are sorted inside each column.
    """
    ncols = n
    m = n if nrows is None else nrows
    if d > m:
        raise ValueError("d exceeds the number of rows")
    rng = np.random.default_rng(seed)
    if 4 * d > m:
        # dense columns: draw without replacement column by column
        rows = np.stack([np.sort(rng.choice(m, d, replace=False)) for _ in range(ncols)]) if ncols else np.zeros((0, d), np.int64)
        nnz = ncols * d
        return Csx(m, ncols, np.arange(0, nnz + 1, d, dtype=np.int64), rows.reshape(-1).astype(np.int32),
                   _values(rng, nnz, values), "csc")
    rows = rng.integers(0, m, size=(ncols, d), dtype=np.int64)
    rows.sort(axis=1)
    while True:
        bad = np.nonzero(np.any(rows[:, 1:] == rows[:, :-1], axis=1))[0] if d > 1 else np.zeros(0, np.int64)
        if bad.size == 0:
            break
        redraw = rng.integers(0, m, size=(bad.size, d), dtype=np.int64)
        redraw.sort(axis=1)
        rows[bad] = redraw
    nnz = ncols * d
    ptr = np.arange(0, nnz + 1, d, dtype=np.int64)
    idx = rows.reshape(-1).astype(np.int32)
    val = _values(rng, nnz, values)
    return Csx(m, ncols, ptr, idx, val, "csc")


def er_problem(n: int, d: int, seed_a: int, seed_b: int | None, values: str = "uniform"):
    """(A in CSC, B in CSR) for C = A*B with ER inputs.

    With ``seed_b is None`` B is A itself (C = A*A), stored as CSR.
    """
    a = er_csc(n, d, seed_a, values=values)
    if seed_b is None:
        b = csc_to_csr(a)
    else:
        b = csc_to_csr(er_csc(n, d, seed_b, values=values))
    return a, b


def identity(n: int, fmt: str) -> Csx:
    ptr = np.arange(n + 1, dtype=np.int64)
    return Csx(n, n, ptr, np.arange(n, dtype=np.int32), np.ones(n), fmt)


def random_sparse(
    m: int,
    n: int,
    density: float,
    seed: int,
    fmt: str,
    values: str = "uniform",
    dense_rows: tuple = (),
    dense_cols: tuple = (),
    empty_rows: tuple = (),
    empty_cols: tuple = (),
) -> Csx:
    """Bernoulli(density) pattern with optional full/empty rows and columns."""
    rng = np.random.default_rng(seed)
    mask = rng.random((m, n)) < density
    for r in dense_rows:
        mask[r, :] = True
    for c in dense_cols:
        mask[:, c] = True
    for r in empty_rows:
        mask[r, :] = False
    for c in empty_cols:
        mask[:, c] = False
    if fmt == "csc":
        cc, rr = np.nonzero(mask.T)  # column-major order
        val = _values(rng, rr.size, values)
        ptr, idx, val = _compress(n, cc, rr, val)
        return Csx(m, n, ptr, idx, val, "csc")
    rr, cc = np.nonzero(mask)
    val = _values(rng, rr.size, values)
    ptr, idx, val = _compress(m, rr, cc, val)
    return Csx(m, n, ptr, idx, val, "csr")


def rmat_symmetric(
    scale: int,
    edge_factor: int,
    seed_edges: int = 12345,
    seed_perm: int | None = 5,
    seed_vals: int = 6,
    abcd=(0.57, 0.19, 0.19, 0.05),
) -> Csx:
    """Symmetric R-MAT adjacency matrix (CSR; its arrays are also its CSC).

    Edges: ``rng = default_rng(seed_edges)``; for each of ``scale`` levels one
    uniform draw per edge picks the quadrant (row bit set when u >= a+b; column
    bit set when a <= u < a+b or u >= a+b+c).  The pattern is symmetrised and
    deduplicated, self-loops are kept, a seeded vertex permutation is applied
    (``seed_perm=None`` skips it), and each unordered pair gets one U[0,1)
    value mirrored to both triangles so the matrix is numerically symmetric.
    """
    a, b, c, _ = abcd
    n = 1 << scale
    m_edges = edge_factor * n
    rng = np.random.default_rng(seed_edges)
    row = np.zeros(m_edges, dtype=np.int64)
    col = np.zeros(m_edges, dtype=np.int64)
    for lvl in range(scale):
        u = rng.random(m_edges)
        rbit = u >= a + b
        cbit = ((u >= a) & (u < a + b)) | (u >= a + b + c)
        row |= rbit.astype(np.int64) << lvl
        col |= cbit.astype(np.int64) << lvl
    del u, rbit, cbit
    if seed_perm is not None:
        perm = np.random.default_rng(seed_perm).permutation(n).astype(np.int64)
        row = perm[row]
        col = perm[col]
    lo = np.minimum(row, col)
    hi = np.maximum(row, col)
    del row, col
    pair = np.unique(lo * n + hi)  # unordered pairs, sorted
    lo = pair // n
    hi = pair % n
    del pair
    pv = np.random.default_rng(seed_vals).random(lo.size)
    off = lo != hi
    rows = np.concatenate([lo, hi[off]])
    cols = np.concatenate([hi, lo[off]])
    vals = np.concatenate([pv, pv[off]])
    del lo, hi, pv, off
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    rows = rows[order]
    cols = cols[order].astype(np.int32)
    vals = vals[order]
    counts = np.bincount(rows, minlength=n).astype(np.int64)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    return Csx(n, n, ptr, cols, vals, "csr")


def batched_er_sizes(count: int = 512, seed: int = 4, lo_log2: int = 10, hi_log2: int = 17):
    """Sizes of the batched ER workload: n_i log-uniform in [2^lo, 2^hi],
    d_i uniform in {2..32}.  All n_i are drawn first, then all d_i."""
    rng = np.random.default_rng(seed)
    n = np.floor(np.exp(rng.uniform(math.log(2.0**lo_log2), math.log(2.0**hi_log2 + 1), count))).astype(np.int64)
    n = np.clip(n, 2**lo_log2, 2**hi_log2)
    d = rng.integers(2, 33, count).astype(np.int64)
    return n, d


def batched_er_problems(count: int = 512, seed: int = 4, values: str = "signed", lo_log2: int = 10, hi_log2: int = 17):
    """Yield (A_i CSC, B_i CSR) for the batched workload; A_i seed 1000+i,
    B_i seed 2000+i, values U[-1,1) by default."""
    n, d = batched_er_sizes(count, seed, lo_log2, hi_log2)
    for i in range(count):
        yield er_problem(int(n[i]), int(d[i]), 1000 + i, 2000 + i, values=values)


def amg_problem(nx: int, omega: float = 2.0 / 3.0):
    """3-D 7-point Laplacian on an nx^3 grid and its smoothed-aggregation
    prolongator from aligned 2x2x2 aggregates.

    A: diagonal 6, -1 for each in-grid neighbour (Dirichlet boundary).
    P0(i, agg(i)) = 1; P = (I - omega D^-1 A) P0 with D = diag(A) = 6.
    Entry by entry that is, for fine node i and aggregate J,
        P(i, J) = [agg(i) = J] (1 - omega) + (omega / 6) * #{grid neighbours j of i with agg(j) = J},
    which needs no matrix product.  Returns (A as CSR, P as CSR); A is
    symmetric so its CSR arrays are also its CSC arrays, and R = P^T in CSC
    is P's CSR arrays read as columns.
    """
    assert nx % 2 == 0
    n = nx**3
    nc = (nx // 2) ** 3
    g = np.arange(n, dtype=np.int64)
    x = g % nx
    y = (g // nx) % nx
    z = g // (nx * nx)
    # neighbour offsets in index order (z-1, y-1, x-1, self, x+1, y+1, z+1)
    offs = [(-nx * nx, z > 0), (-nx, y > 0), (-1, x > 0), (0, None), (1, x < nx - 1), (nx, y < nx - 1), (nx * nx, z < nx - 1)]
    rows, cols, vals = [], [], []
    for o, ok in offs:
        if ok is None:
            rows.append(g)
            cols.append(g)
            vals.append(np.full(n, 6.0))
        else:
            s = g[ok]
            rows.append(s)
            cols.append(s + o)
            vals.append(np.full(s.size, -1.0))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    order = np.lexsort((cols, rows))
    ptr, idx, val = _compress(n, rows[order], cols[order], vals[order])
    A = Csx(n, n, ptr, idx, val, "csr")

    ncx = nx // 2

    def agg_of(xx, yy, zz):
        return (zz // 2) * ncx * ncx + (yy // 2) * ncx + (xx // 2)

    own = agg_of(x, y, z)
    # (i, J) pairs: i's own aggregate once (weight 0 neighbours so far) plus one
    # pair per in-grid neighbour j of i, J = agg(j).
    prow, pcol, isnb = [g], [own], [np.zeros(n, np.int64)]
    nb = [(-1, 0, 0, x > 0), (1, 0, 0, x < nx - 1), (0, -1, 0, y > 0), (0, 1, 0, y < nx - 1), (0, 0, -1, z > 0), (0, 0, 1, z < nx - 1)]
    for dx, dy, dz, ok in nb:
        s = g[ok]
        prow.append(s)
        pcol.append(agg_of(x[ok] + dx, y[ok] + dy, z[ok] + dz))
        isnb.append(np.ones(s.size, np.int64))
    prow = np.concatenate(prow)
    pcol = np.concatenate(pcol)
    isnb = np.concatenate(isnb)
    key = prow * nc + pcol
    uk, inv = np.unique(key, return_inverse=True)
    count = np.bincount(inv, weights=isnb, minlength=uk.size)  # integer-valued
    pr = uk // nc
    pc = uk % nc
    val = np.where(pc == own[pr], 1.0 - omega, 0.0) + (omega / 6.0) * count
    ptr, idx, val = _compress(n, pr, pc.astype(np.int32), val)
    P = Csx(n, nc, ptr, idx, val, "csr")
    return A, P
