"""GPU parity for row-range rounds and rows wider than the tile (column
windows, dense windows), against the CPU oracle."""
import sys

import numpy as np
import pytest

import oracle
from workloads import Csx, er_csc, er_problem, rmat_symmetric

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


def _check(got: dict, ref: dict, precision: str):
    assert np.array_equal(got["rowptr"], ref["rowptr"]), "row pointers"
    assert np.array_equal(got["colidx"], ref["colidx"]), "column indices"
    err = np.abs(got["val"].astype(np.float64) - ref["val"])
    bad = err > TOL[precision] * ref["absval"]
    assert not bad.any(), f"{bad.sum()} values beyond tolerance, worst {np.max(err / np.maximum(ref['absval'], 1e-300))}"


def _run(pb, a, b, precision, tune):
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    return pb.spgemm(A, B, precision=precision, tune=tune).to_host()


def _rows_of(ref: dict, r0: int, r1: int) -> dict:
    s, e = ref["rowptr"][r0], ref["rowptr"][r1]
    return dict(rowptr=ref["rowptr"][r0:r1 + 1] - s, colidx=ref["colidx"][s:e], val=ref["val"][s:e],
                absval=ref["absval"][s:e])


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_rounds_whole_c(pb, precision):
    """A product cut into several rounds by a small tuple budget, written
    into one C by spgemm_numeric."""
    _say(f"ER 20000 d=8, rounds of <= 300000 tuples, {precision}")
    a, b = er_problem(20000, 8, 41, 42, values="signed")
    got = _run(pb, a, b, precision, {"round_tuples": 300_000})
    _check(got, oracle.spgemm(a, b), precision)


def test_rounds_one_at_a_time(pb):
    """Rounds taken one by one through spgemm_numeric_round, each into its
    own buffers with row pointers starting at 0."""
    import torch

    _say("ER 12000 d=6, per-round output")
    a, b = er_problem(12000, 6, 43, 44, values="signed")
    ref = oracle.spgemm(a, b)
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    tune = {"round_tuples": 100_000, "tile_tuples": 2048}
    nsym = pb.spgemm_symbolic(A, B, "f64", tune)
    sym = torch.empty(nsym, dtype=torch.uint8, device="cuda")
    plan = pb.spgemm_symbolic(A, B, "f64", tune, sym_ws=sym)
    rb, fl = pb.spgemm_plan_rounds(plan)
    assert len(rb) >= 4 and rb[0] == 0 and rb[-1] == a.nrows and sum(fl) == plan.info()["slots"]
    assert max(fl) <= 100_000
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    for r in range(len(fl)):
        nrows = rb[r + 1] - rb[r]
        rp = torch.empty(nrows + 1, dtype=torch.int64, device="cuda")
        ci = torch.empty(max(fl[r], 1), dtype=torch.int32, device="cuda")
        cv = torch.empty(max(fl[r], 1), dtype=torch.float64, device="cuda")
        nnz = pb.spgemm_numeric_round(plan, A, B, r, ws, rp, ci, cv)
        got = dict(rowptr=rp.cpu().numpy(), colidx=ci[:nnz].cpu().numpy(), val=cv[:nnz].cpu().numpy())
        _check(got, _rows_of(ref, rb[r], rb[r + 1]), "f64")
    plan.close()


def test_round_budget_invariance(pb):
    """C does not depend on the round budget: bit-equal structure for every
    budget, including one bin per round."""
    _say("ER 3000 d=5, budgets 0 / 50000 / 1")
    a, b = er_problem(3000, 5, 45, 46)
    outs = [_run(pb, a, b, "f64", {"round_tuples": rt, "tile_tuples": 512}) for rt in (0, 50_000, 1)]
    for o in outs[1:]:
        assert np.array_equal(o["rowptr"], outs[0]["rowptr"]) and np.array_equal(o["colidx"], outs[0]["colidx"])
    _check(outs[2], oracle.spgemm(a, b), "f64")


@pytest.mark.parametrize("scale,tile,precision", [(11, 4096, "f64"), (12, 1024, "f64"), (13, 4096, "f32c"),
                                                  (13, 2048, "f64")])
def test_rmat_wide_rows(pb, scale, tile, precision):
    """R-MAT A*A: hub rows far wider than the tile go through the column
    windows; windows above the tile through the dense accumulator."""
    _say(f"R-MAT scale {scale} A*A, tile {tile}, {precision}")
    a = rmat_symmetric(scale, 16)
    ac = a.transpose_view()  # symmetric: the CSR arrays are also A's CSC
    got = _run(pb, ac, a, precision, {"tile_tuples": tile})
    _check(got, oracle.spgemm(ac, a), precision)


def test_rmat_wide_rows_with_rounds(pb):
    _say("R-MAT scale 12 A*A, rounds of <= 2M tuples")
    a = rmat_symmetric(12, 16)
    ac = a.transpose_view()
    got = _run(pb, ac, a, "f64", {"round_tuples": 2_000_000})
    _check(got, oracle.spgemm(ac, a), "f64")


def _a_with_full_rows(m, k, full_rows, density, seed):
    """A (CSC) Bernoulli(density) with a few full rows: their C rows are wide."""
    rng = np.random.default_rng(seed)
    dm = rng.random((m, k)) < density
    dm[list(full_rows), :] = True
    return _csc_from_mask(dm, rng.uniform(-1, 1, size=(m, k)) * dm)


def _b_d_per_row(k, n, d, seed):
    """B (k x n, CSR) with exactly d distinct uniform columns per row, built
    without a dense mask (n may be large)."""
    return er_csc(k, d, seed, nrows=n, values="signed").transpose_view()


def _csc_from_mask(mask, vals):
    m, k = mask.shape
    ptr = np.zeros(k + 1, np.int64)
    idx, val = [], []
    for j in range(k):
        rows = np.nonzero(mask[:, j])[0]
        idx.append(rows.astype(np.int32))
        val.append(vals[rows, j])
        ptr[j + 1] = ptr[j] + len(rows)
    return Csx(m, k, ptr, np.concatenate(idx), np.concatenate(val).astype(np.float64), "csc")


def test_wide_rows_many_windows(pb):
    """n = 2^20 columns: a wide row is split into 256 windows of 4096."""
    _say("wide rows over n=2^20 columns (256 windows)")
    m, k, n = 300, 2000, 1 << 20
    a = _a_with_full_rows(m, k, [0, 7, 150, 299], 0.01, 51)
    b = _b_d_per_row(k, n, 32, 52)
    got = _run(pb, a, b, "f64", {"tile_tuples": 1024})
    _check(got, oracle.spgemm(a, b), "f64")


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_dense_window_single_column(pb, precision):
    """Every tuple of a wide row lands on one column: one dense window whose
    accumulator takes all adds on one address (and a cancellation)."""
    _say(f"dense window, one hot column, {precision}")
    m, k, n = 40, 6000, 100
    rng = np.random.default_rng(61)
    mask = rng.random((m, k)) < 0.05
    mask[3, :] = True
    vals = rng.uniform(0.5, 1.0, size=(m, k)) * mask
    a = _csc_from_mask(mask, vals)
    # B: column 0 in every row, plus a few random columns; values +-1 so
    # row 3, column 0 sums to (near) zero but stays stored
    bptr = np.zeros(k + 1, np.int64)
    bidx, bval = [], []
    for r in range(k):
        cols = np.unique(np.concatenate([[0], rng.integers(1, n, 2)])).astype(np.int32)
        bidx.append(cols)
        v = rng.uniform(-1, 1, len(cols))
        v[0] = 1.0 if r % 2 == 0 else -1.0
        bval.append(v)
        bptr[r + 1] = bptr[r] + len(cols)
    b = Csx(k, n, bptr, np.concatenate(bidx), np.concatenate(bval), "csr")
    got = _run(pb, a, b, precision, {"tile_tuples": 512})
    _check(got, oracle.spgemm(a, b), precision)


def test_wide_window_beyond_dense_is_rejected(pb):
    """n > 2^22 makes windows wider than the dense accumulator; a wide row
    whose tuples pile onto one column then cannot be done: the numeric step
    reports PB_ERR_UNSUPPORTED (and a spread-out wide row still works)."""
    _say("n = 2^23: spread wide row works, clustered one is rejected")
    m, k, n = 8, 3000, 1 << 23
    rng = np.random.default_rng(71)
    mask = np.zeros((m, k), bool)
    mask[2, :] = True
    a = _csc_from_mask(mask, rng.uniform(0.5, 1, size=(m, k)) * mask)
    spread = _b_d_per_row(k, n, 3, 72)
    got = _run(pb, a, spread, "f64", {"tile_tuples": 1024})
    _check(got, oracle.spgemm(a, spread), "f64")
    one = Csx(k, n, np.arange(k + 1, dtype=np.int64), np.zeros(k, np.int32), np.ones(k), "csr")
    with pytest.raises(pb.PbError) as ei:
        _run(pb, a, one, "f64", {"tile_tuples": 1024})
    assert ei.value.name == "PB_ERR_UNSUPPORTED"
