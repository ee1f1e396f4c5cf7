"""spgemm_numeric_noalloc: the numeric step on the library's per-GPU device
scratch, with no workspace argument and no allocation, against
spgemm_numeric on the same plan (and against the oracle): two calls in a
row on one GPU, the second with a smaller product, so the second finds the
first one's contents in the scratch."""
import sys

import numpy as np
import pytest

import oracle
from workloads import er_problem

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


def _plan(pb, torch, A, B, precision, tune=None):
    nsym = pb.spgemm_symbolic(A, B, precision, tune)
    sym = torch.empty(nsym, dtype=torch.uint8, device="cuda")
    return pb.spgemm_symbolic(A, B, precision, tune, sym_ws=sym)


def _outputs(torch, m, flop, precision):
    vdt = torch.float64 if precision == "f64" else torch.float32
    return (torch.full((m + 1,), -1, dtype=torch.int64, device="cuda"),
            torch.full((max(flop, 1),), -1, dtype=torch.int32, device="cuda"),
            torch.full((max(flop, 1),), float("nan"), dtype=vdt, device="cuda"))


def _check_pair(a, b, got, base, precision):
    rp, ci, cv = (x.cpu().numpy() for x in got)
    brp, bci, bcv = (x.cpu().numpy() for x in base)
    nnz = int(brp[-1])
    assert np.array_equal(rp, brp), "row pointers differ from spgemm_numeric"
    assert np.array_equal(ci[:nnz], bci[:nnz]), "columns differ from spgemm_numeric"
    ref = oracle.spgemm(a, b)
    assert np.array_equal(rp, ref["rowptr"]) and np.array_equal(ci[:nnz], ref["colidx"])
    bound = TOL[precision] * ref["absval"]
    assert np.all(np.abs(cv[:nnz].astype(np.float64) - ref["val"]) <= bound), "values vs oracle"
    assert np.all(np.abs(cv[:nnz].astype(np.float64) - bcv[:nnz].astype(np.float64)) <= 2 * bound), \
        "values vs spgemm_numeric"


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_noalloc_matches_numeric_two_calls(pb, precision):
    import torch

    cases = [(er_problem(20000, 9, 301, 302, values="signed"), None),
             (er_problem(3000, 4, 303, 304, values="signed"), None)]
    for i, ((a, b), tune) in enumerate(cases):
        _say(f"no-alloc call {i}: n={a.nrows} {precision}")
        A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
        plan = _plan(pb, torch, A, B, precision, tune)
        assert plan.workspace_bytes <= pb.NOALLOC_SCRATCH_BYTES
        ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
        base = _outputs(torch, a.nrows, plan.flop, precision)
        nnz0 = pb.spgemm_numeric(plan, A, B, ws, *base)
        got = _outputs(torch, a.nrows, plan.flop, precision)
        nnz1 = pb.spgemm_numeric_noalloc(plan, A, B, *got)
        assert nnz0 == nnz1
        _check_pair(a, b, got, base, precision)
        plan.close()


def test_noalloc_rounds_plan(pb):
    """A plan of several rounds (and a row wider than the tile) runs all its
    rounds in the scratch."""
    import torch

    from workloads import random_sparse

    _say("no-alloc rounds plan")
    a = random_sparse(3000, 900, 0.004, 305, "csc", values="signed", dense_rows=(7,))
    b = random_sparse(900, 2500, 0.004, 306, "csr", values="signed")
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    plan = _plan(pb, torch, A, B, "f64", {"tile_tuples": 512, "round_tuples": 20000})
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    base = _outputs(torch, a.nrows, plan.flop, "f64")
    pb.spgemm_numeric(plan, A, B, ws, *base)
    got = _outputs(torch, a.nrows, plan.flop, "f64")
    pb.spgemm_numeric_noalloc(plan, A, B, *got)
    _check_pair(a, b, got, base, "f64")
    plan.close()


def test_noalloc_rejects_large_plan(pb):
    import torch

    _say("no-alloc rejects a plan above the scratch size")
    a, b = er_problem(1 << 17, 16, 307, 308)
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    plan = _plan(pb, torch, A, B, "f64")
    assert plan.workspace_bytes > pb.NOALLOC_SCRATCH_BYTES
    out = _outputs(torch, a.nrows, plan.flop, "f64")
    with pytest.raises(pb.PbError) as ei:
        pb.spgemm_numeric_noalloc(plan, A, B, *out)
    assert ei.value.name == "PB_ERR_WORKSPACE"
    assert int(out[0][0].item()) == -1  # nothing ran
    plan.close()
