"""Properties of the seeded input generators (CPU only)."""
import numpy as np
import pytest

from workloads import amg_problem, batched_er_sizes, csc_to_csr, csr_to_csc, er_csc, er_problem, rmat_symmetric


def test_er_exact_d_distinct_sorted():
    a = er_csc(5000, 7, seed=3)
    a.check()
    assert np.all(np.diff(a.ptr) == 7)
    rows = a.idx.reshape(5000, 7).astype(np.int64)
    assert np.all(np.diff(rows, axis=1) > 0)
    # roughly uniform row usage
    counts = np.bincount(a.idx, minlength=5000)
    assert abs(counts.mean() - 7) < 1e-9 and counts.std() < 4


def test_er_deterministic_in_seed():
    a1 = er_csc(1000, 4, seed=9)
    a2 = er_csc(1000, 4, seed=9)
    a3 = er_csc(1000, 4, seed=10)
    assert np.array_equal(a1.idx, a2.idx) and np.array_equal(a1.val, a2.val)
    assert not np.array_equal(a1.idx, a3.idx)


def test_format_roundtrip():
    a, b = er_problem(3000, 5, 1, 2)
    a.check()
    b.check()
    back = csr_to_csc(csc_to_csr(a))
    assert np.array_equal(back.ptr, a.ptr) and np.array_equal(back.idx, a.idx) and np.array_equal(back.val, a.val)


def test_rmat_small_symmetric_no_duplicates():
    g = rmat_symmetric(10, 8, seed_edges=1, seed_perm=2, seed_vals=3)
    g.check()
    n = g.nrows
    rows = np.repeat(np.arange(n), np.diff(g.ptr))
    key = rows * n + g.idx
    assert np.unique(key).size == key.size
    kt = g.idx.astype(np.int64) * n + rows
    order = np.argsort(kt)
    assert np.array_equal(np.sort(key), kt[order])
    # numerically symmetric: value of (i, j) equals value of (j, i)
    assert np.array_equal(g.val[np.argsort(key)], g.val[order])
    deg = np.diff(g.ptr)
    assert deg.max() > 8 * deg.mean()  # skewed degrees


def test_amg_closed_forms():
    nx = 16
    n = nx**3
    A, P = amg_problem(nx)
    A.check()
    P.check()
    assert A.nnz == n + 6 * nx * nx * (nx - 1)
    assert P.nnz == 4 * n - 6 * nx * nx  # own aggregate + one per in-grid outward direction
    assert P.ncols == (nx // 2) ** 3
    rowsum = np.add.reduceat(P.val, P.ptr[:-1])
    g = np.arange(n)
    x, y, z = g % nx, (g // nx) % nx, g // (nx * nx)
    interior = (x > 0) & (x < nx - 1) & (y > 0) & (y < nx - 1) & (z > 0) & (z < nx - 1)
    assert np.allclose(rowsum[interior], 1.0, rtol=0, atol=1e-15)
    assert np.all(rowsum[~interior] < 1.0)
    vals = np.unique(np.round(P.val, 15))
    assert np.allclose(sorted(vals), [1.0 / 9.0, 2.0 / 3.0], atol=1e-15)
    # symmetric A: CSR arrays equal the CSC arrays
    At = csr_to_csc(A)
    assert np.array_equal(At.ptr, A.ptr) and np.array_equal(At.idx, A.idx) and np.array_equal(At.val, A.val)


def test_batched_sizes():
    n, d = batched_er_sizes(512, 4)
    assert n.min() >= 2**10 and n.max() <= 2**17
    assert d.min() >= 2 and d.max() <= 32
    # log-uniform: about half the problems below the geometric midpoint 2^13.5
    assert 0.35 < np.mean(n < 2**13.5) < 0.65


@pytest.mark.slow
def test_amg_full_counts():
    A, P = amg_problem(128)
    assert A.nnz == 14_581_760 and P.nnz == 8_290_304 and np.diff(P.ptr).max() == 4
