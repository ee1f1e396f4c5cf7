"""Output and operand variants of the product on the same kernels, against
the oracle: C returned in CSC (as C^T = B^T A^T in CSR), A*A^T for a
rectangular A, and a tall-skinny B (a few columns, the shape of a batch of
graph frontiers)."""
import sys

import numpy as np
import pytest

import oracle
from workloads import Csx, er_csc, er_problem, random_sparse

pytestmark = pytest.mark.gpu
TOL = {"f64": 1e-12, "f32c": 1e-6}


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pb():
    import torch

    assert torch.cuda.is_available()
    import paper_2002_11302_amd as pbm

    pbm.load()
    return pbm


def _to_csc(m, n, rowptr, colidx, vals):
    """CSR arrays of an m x n matrix -> CSC arrays (stable in rows)."""
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    order = np.lexsort((rows, colidx))
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ptr, colidx.astype(np.int64) + 1, 1)
    return np.cumsum(ptr), rows[order], [v[order] for v in vals]


def _check(got_ptr, got_idx, got_val, ref_ptr, ref_idx, ref_val, ref_abs, precision):
    assert np.array_equal(got_ptr, ref_ptr), "pointers"
    assert np.array_equal(got_idx, ref_idx), "indices"
    err = np.abs(got_val.astype(np.float64) - ref_val)
    assert np.all(err <= TOL[precision] * ref_abs), f"values: worst {np.max(err / np.maximum(ref_abs, 1e-300)):.3e}"


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_c_in_csc(pb, precision):
    _say(f"C = A*B returned in CSC, rectangular, {precision}")
    a = random_sparse(300, 200, 0.03, 51, "csc", values="signed", dense_cols=(7,), empty_rows=(5,))
    b = random_sparse(200, 450, 0.02, 52, "csr", values="signed", dense_rows=(11,), empty_cols=(3, 4))
    c = pb.spgemm_csc(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b), precision=precision)
    assert (c.nrows, c.ncols) == (a.nrows, b.ncols)
    ref = oracle.spgemm(a, b)
    ptr, idx, (val, absval) = _to_csc(a.nrows, b.ncols, ref["rowptr"], ref["colidx"], (ref["val"], ref["absval"]))
    _check(c.ptr.cpu().numpy(), c.idx.cpu().numpy(), c.val.cpu().numpy(), ptr, idx, val, absval, precision)


def test_a_times_a_transpose(pb):
    """A*A^T for a 3000 x 1000 A in CSC: A^T in CSR is A's own arrays."""
    _say("A*A^T, A 3000 x 1000 ER")
    a = er_csc(1000, 6, 61, nrows=3000)
    at_csr = Csx(a.ncols, a.nrows, a.ptr, a.idx, a.val, "csr")
    A = pb.DeviceCsx.from_host(a)
    got = pb.spgemm(A, A.transpose_view()).to_host()
    ref = oracle.spgemm(a, at_csr)
    _check(got["rowptr"], got["colidx"], got["val"], ref["rowptr"], ref["colidx"], ref["val"], ref["absval"], "f64")
    # A*A^T is symmetric: its CSR arrays are its CSC arrays
    ptr, idx, (val,) = _to_csc(a.nrows, a.nrows, got["rowptr"], got["colidx"], (got["val"],))
    assert np.array_equal(ptr, got["rowptr"]) and np.array_equal(idx, got["colidx"])


@pytest.mark.parametrize("ncols", [1, 8, 64])
def test_tall_skinny_b(pb, ncols):
    """A square graph-like A times an n x ncols B with a few entries per row."""
    _say(f"A (ER 2^14, d=8) * B (2^14 x {ncols})")
    a, _ = er_problem(1 << 14, 8, 71, None)
    b = random_sparse(1 << 14, ncols, min(1.0, 3.0 / ncols), 72, "csr")
    got = pb.spgemm(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)).to_host()
    ref = oracle.spgemm(a, b)
    _check(got["rowptr"], got["colidx"], got["val"], ref["rowptr"], ref["colidx"], ref["val"], ref["absval"], "f64")
