"""GPU parity for the AMG Galerkin chain Ac = R (A P): two chained products.

A is the 7-point Laplacian (symmetric, so its CSR arrays are its CSC
arrays); P is the smoothed-aggregation prolongator in CSR; R = P^T in CSC
is P's CSR arrays read as columns.  T = A*P is emitted as CSR and feeds the
second product directly.
"""
import sys

import numpy as np
import pytest

import oracle
from workloads import Csx, amg_problem

pytestmark = pytest.mark.gpu


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


def _check(got: dict, ref: dict, tol: float):
    assert np.array_equal(got["rowptr"], ref["rowptr"])
    assert np.array_equal(got["colidx"], ref["colidx"])
    err = np.abs(got["val"].astype(np.float64) - ref["val"])
    assert np.all(err <= tol * ref["absval"]), float(np.max(err / np.maximum(ref["absval"], 1e-300)))


@pytest.mark.parametrize("precision,tol", [("f64", 1e-12), ("f32c", 1e-6)])
@pytest.mark.parametrize("nx", [8, 24])
def test_galerkin_chain(pb, nx, precision, tol):
    import torch

    _say(f"AMG R*(A*P) nx={nx} {precision}")
    A, P = amg_problem(nx)
    a_csc = Csx(A.nrows, A.ncols, A.ptr, A.idx, A.val, "csc")  # symmetric
    t_ref = oracle.spgemm(a_csc, P)
    T = pb.spgemm(pb.DeviceCsx.from_host(a_csc), pb.DeviceCsx.from_host(P), precision=precision)
    _check(T.to_host(), t_ref, tol)
    # second product: R = P^T in CSC (P's CSR arrays) times T in CSR
    t_dev = pb.DeviceCsx(T.nrows, T.ncols, T.rowptr, T.colidx, T.val.to(torch.float64))
    R = pb.DeviceCsx.from_host(P).transpose_view()
    Ac = pb.spgemm(R, t_dev, precision=precision)
    t_host = Csx(t_ref["nrows"], t_ref["ncols"], t_ref["rowptr"], t_ref["colidx"], t_ref["val"], "csr")
    ac_ref = oracle.spgemm(P.transpose_view(), t_host)
    # the second product's inputs are the first product's (rounded) outputs:
    # allow the first stage's error to propagate through |R||T|
    got = Ac.to_host()
    assert np.array_equal(got["rowptr"], ac_ref["rowptr"])
    assert np.array_equal(got["colidx"], ac_ref["colidx"])
    err = np.abs(got["val"].astype(np.float64) - ac_ref["val"])
    assert np.all(err <= 4 * tol * ac_ref["absval"])
    # Galerkin operator of a symmetric A is symmetric in structure
    n_c = Ac.nrows
    rows = np.repeat(np.arange(n_c), np.diff(got["rowptr"]))
    k1 = rows * n_c + got["colidx"]
    k2 = got["colidx"].astype(np.int64) * n_c + rows
    assert np.array_equal(np.sort(k1), np.sort(k2))


def test_galerkin_full_size(pb):
    """128^3 grid: both products of the chain against the oracle, whole."""
    import torch

    _say("AMG R*(A*P) nx=128 f64")
    A, P = amg_problem(128)
    a_csc = Csx(A.nrows, A.ncols, A.ptr, A.idx, A.val, "csc")
    T = pb.spgemm(pb.DeviceCsx.from_host(a_csc), pb.DeviceCsx.from_host(P))
    t_ref = oracle.spgemm(a_csc, P)
    _check(T.to_host(), t_ref, 1e-12)
    t_dev = pb.DeviceCsx(T.nrows, T.ncols, T.rowptr, T.colidx, T.val)
    Ac = pb.spgemm(pb.DeviceCsx.from_host(P).transpose_view(), t_dev)
    t_host = Csx(t_ref["nrows"], t_ref["ncols"], t_ref["rowptr"], t_ref["colidx"], t_ref["val"], "csr")
    ac_ref = oracle.spgemm(P.transpose_view(), t_host)
    got = Ac.to_host()
    assert np.array_equal(got["rowptr"], ac_ref["rowptr"]) and np.array_equal(got["colidx"], ac_ref["colidx"])
    assert np.all(np.abs(got["val"] - ac_ref["val"]) <= 4e-12 * ac_ref["absval"])
