"""GPU parity for the full-size R-MAT product C = A*A (scale 20, edge
factor 16): 7e10 tuples and 2.4e10 entries of C, so the product runs in
row-range rounds into one reused buffer.  The oracle computes sampled rows
(the heaviest hub rows and random rows) and the lightest round (every row
of it while its multiplications stay under 2.5e9, row pointers included)
exactly; every round is also checked for properties that hold at any
size."""
import os
import sys

import numpy as np
import pytest

import oracle
from workloads import rmat_symmetric

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
TOL = {"f64": 1e-12, "f32c": 1e-6}
ROUND_TUPLES = 1 << 32


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch

    assert torch.cuda.is_available()
    import paper_2002_11302_amd as pb

    pb.load()
    _say("R-MAT scale 20 ef 16: generating")
    a = rmat_symmetric(20, 16)
    ac = a.transpose_view()
    deg = np.diff(a.ptr)
    rowflop = np.bincount(np.repeat(np.arange(a.nrows), deg), weights=deg[a.idx].astype(np.float64),
                          minlength=a.nrows)
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([np.argsort(rowflop)[-24:], rng.integers(0, a.nrows, 40)]))
    _say(f"oracle on {rows.size} sampled rows ({int(rowflop[rows].sum())} flop)")
    ref = oracle.spgemm_rows(ac, a, rows, nthreads=len(os.sched_getaffinity(0)))
    return pb, torch, a, ac, rows, ref, rowflop


_BLOCK = {}


def _block_ref(ac, a, rowflop, r0, r1, nth):
    """Oracle rows [r0, r1') where r1' <= r1 keeps the block's
    multiplications under 2.5e9 (at least one row)."""
    key = (r0, r1)
    if key not in _BLOCK:
        cum = np.cumsum(rowflop[r0:r1])
        nrow = max(1, int(np.searchsorted(cum, 2.5e9, side="right")))
        rows = np.arange(r0, r0 + nrow, dtype=np.int64)
        _say(f"oracle on rows [{r0}, {r0 + nrow}) of the lightest round ({int(cum[nrow - 1])} flop)")
        _BLOCK[key] = (rows, oracle.spgemm_rows(ac, a, rows, nthreads=nth))
    return _BLOCK[key]


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_rmat_scale20_rounds(setup, precision):
    pb, torch, a, ac, rows, ref, rowflop = setup
    A, B = pb.DeviceCsx.from_host(ac), pb.DeviceCsx.from_host(a)
    tune = {"round_tuples": ROUND_TUPLES}
    nsym = pb.spgemm_symbolic(A, B, precision, tune)
    sym = torch.empty(nsym, dtype=torch.uint8, device="cuda")
    plan = pb.spgemm_symbolic(A, B, precision, tune, sym_ws=sym)
    rb, fl = pb.spgemm_plan_rounds(plan)
    assert rb[0] == 0 and rb[-1] == a.nrows and sum(fl) == plan.info()["slots"] >= plan.flop
    _say(f"{precision}: flop {plan.flop}, {len(fl)} rounds, workspace {plan.workspace_bytes / 1e9:.1f} GB")
    light = int(np.argmin(fl))
    brows, bref = _block_ref(ac, a, rowflop, rb[light], rb[light + 1], len(os.sched_getaffinity(0)))
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    maxrows = max(rb[i + 1] - rb[i] for i in range(len(fl)))
    rp = torch.empty(maxrows + 1, dtype=torch.int64, device="cuda")
    ci = torch.empty(max(fl), dtype=torch.int32, device="cuda")
    cv = torch.empty(max(fl), dtype=torch.float64 if precision == "f64" else torch.float32, device="cuda")
    seen = 0
    for r in range(len(fl)):
        nnz = pb.spgemm_numeric_round(plan, A, B, r, ws, rp, ci, cv)
        nrows = rb[r + 1] - rb[r]
        assert 0 <= nnz <= fl[r]
        p = rp[: nrows + 1]
        assert int(p[0]) == 0 and int(p[-1]) == nnz and bool(torch.all(p[1:] >= p[:-1]))
        if precision == "f64" and nnz > 1:
            # columns strictly increase inside every row of the round
            c = ci[:nnz].to(torch.int64)
            inc = c[1:] > c[:-1]
            starts = torch.zeros(nnz, dtype=torch.bool, device="cuda")
            inner = p[1:-1]
            starts[inner[inner < nnz]] = True
            assert bool(torch.all(inc | starts[1:])), f"round {r}: unsorted columns"
        sel = rows[(rows >= rb[r]) & (rows < rb[r + 1])]
        if sel.size:
            h = p.cpu().numpy()
            for row in sel:
                s_ = int(np.searchsorted(rows, row))
                want_c = ref["idx"][ref["ptr"][s_]:ref["ptr"][s_ + 1]]
                want_v = ref["val"][ref["ptr"][s_]:ref["ptr"][s_ + 1]]
                nrm = ref["absval"][ref["ptr"][s_]:ref["ptr"][s_ + 1]]
                g0, g1 = int(h[row - rb[r]]), int(h[row - rb[r] + 1])
                got_c = ci[g0:g1].cpu().numpy()
                got_v = cv[g0:g1].cpu().numpy().astype(np.float64)
                assert np.array_equal(got_c, want_c), f"row {row}: structure"
                assert np.all(np.abs(got_v - want_v) <= TOL[precision] * nrm), f"row {row}: values"
                seen += 1
        if r == light:
            # a block of consecutive rows at the round's start: row
            # pointers (relative to the block's first row) and every entry
            h = p.cpu().numpy()
            g0 = int(h[0])
            g1 = int(h[brows.size])
            assert np.array_equal(h[: brows.size + 1] - g0, bref["ptr"]), f"round {r}: row pointers of the block"
            assert np.array_equal(ci[g0:g1].cpu().numpy(), bref["idx"]), f"round {r}: columns of the block"
            gv = cv[g0:g1].cpu().numpy().astype(np.float64)
            assert np.all(np.abs(gv - bref["val"]) <= TOL[precision] * bref["absval"]), f"round {r}: block values"
            whole = "the whole round" if brows.size == nrows else f"{brows.size} of its {nrows} rows"
            _say(f"{precision}: round {r}: {whole}, {g1 - g0} entries, equal the oracle")
        if r % 4 == 0:
            _say(f"{precision}: round {r + 1}/{len(fl)} ok")
    assert seen == rows.size
    plan.close()
