"""GPU parity over the scale x edge-factor grid of the sweep (ER A*B and
R-MAT A*A, the paper's Section 5 performance figures over scales and edge
factors).  Small scales of the grid are compared with the oracle entry by
entry; the largest sweep points (ER scale 22 with 32 nonzeros per column,
2^32 tuples; R-MAT scale 18 edge factor 16 in row-range rounds) on sampled
rows, with the CSR invariants checked on all of C."""
import os
import sys

import numpy as np
import pytest

import oracle
from workloads import er_problem, rmat_symmetric

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


def _inputs(family, scale, ef):
    if family == "er":
        return er_problem(1 << scale, ef, 2, 3)
    r = rmat_symmetric(scale, ef)
    return r.transpose_view(), r  # symmetric: the CSR arrays are also A's CSC


def _check_whole(got, ref, precision):
    assert np.array_equal(got["rowptr"], ref["rowptr"]), "row pointers"
    assert np.array_equal(got["colidx"], ref["colidx"]), "column indices"
    err = np.abs(got["val"].astype(np.float64) - ref["val"])
    bad = err > TOL[precision] * ref["absval"]
    assert not bad.any(), f"{bad.sum()} values beyond tolerance"


def _check_rows(rows, ref, get_row, precision):
    for s_, r in enumerate(rows):
        want_c = ref["idx"][ref["ptr"][s_]:ref["ptr"][s_ + 1]]
        want_v = ref["val"][ref["ptr"][s_]:ref["ptr"][s_ + 1]]
        nrm = ref["absval"][ref["ptr"][s_]:ref["ptr"][s_ + 1]]
        got_c, got_v = get_row(int(r))
        assert np.array_equal(got_c, want_c), f"row {r}: structure"
        assert np.all(np.abs(got_v.astype(np.float64) - want_v) <= TOL[precision] * nrm), f"row {r}: values"


def _sorted_rows_on_device(torch, rp, ci, nrows, step=1 << 18):
    """Columns strictly increase inside every row, checked in row chunks."""
    for r0 in range(0, nrows, step):
        r1 = min(nrows, r0 + step)
        s, e = int(rp[r0]), int(rp[r1])
        if e - s < 2:
            continue
        c = ci[s:e]
        lens = torch.diff(rp[r0:r1 + 1])
        rows = torch.repeat_interleave(torch.arange(r1 - r0, device=c.device), lens)
        ok = (c[1:] > c[:-1]) | (rows[1:] != rows[:-1])
        assert bool(torch.all(ok).item()), f"rows {r0}..{r1}: unsorted columns"


GRID = [("er", s, d) for s in (10, 12, 14) for d in (4, 8, 16, 32)] + \
       [("rmat", s, ef) for s in (10, 12) for ef in (4, 8, 16, 32)] + [("rmat", 14, 4), ("rmat", 14, 16)]


@pytest.mark.parametrize("family,scale,ef", GRID)
def test_sweep_grid_small(pb, family, scale, ef):
    _say(f"sweep grid {family} scale {scale} ef {ef}, FP64, whole C against the oracle")
    a, b = _inputs(family, scale, ef)
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    got = pb.spgemm(A, B, precision="f64").to_host()
    _check_whole(got, oracle.spgemm(a, b), "f64")


@pytest.mark.parametrize("family,scale,ef", [("er", 12, 32), ("rmat", 12, 32)])
def test_sweep_grid_small_f32c(pb, family, scale, ef):
    _say(f"sweep grid {family} scale {scale} ef {ef}, FP32c, whole C against the oracle")
    a, b = _inputs(family, scale, ef)
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    got = pb.spgemm(A, B, precision="f32c").to_host()
    _check_whole(got, oracle.spgemm(a, b), "f32c")


def test_sweep_er_scale22_d32_sampled(pb):
    """The sweep's largest ER point: 2^22 rows, 2^32 tuples, C whole in HBM."""
    import torch

    _say("sweep ER scale 22 d 32 A*B, FP64, sampled rows")
    a, b = _inputs("er", 22, 32)
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    c = pb.spgemm(A, B, precision="f64")
    rp = c.rowptr
    assert int(rp[0]) == 0 and bool(torch.all(rp[1:] >= rp[:-1])) and c.nnz <= (1 << 32)
    _sorted_rows_on_device(torch, rp, c.colidx, a.nrows)
    rng = np.random.default_rng(21)
    rows = np.unique(np.concatenate([[0, a.nrows - 1], rng.integers(0, a.nrows, 512)]))
    ref = oracle.spgemm_rows(a, b, rows, nthreads=len(os.sched_getaffinity(0)))
    h = rp.cpu().numpy()

    def get_row(r):
        return c.colidx[h[r]:h[r + 1]].cpu().numpy(), c.val[h[r]:h[r + 1]].cpu().numpy()

    _check_rows(rows, ref, get_row, "f64")


def test_sweep_rmat_scale18_ef16_rounds_sampled(pb):
    """R-MAT scale 18 edge factor 16 (9.5e9 tuples) in rounds of at most
    2^32 tuples: the heaviest hub rows and random rows against the oracle."""
    import torch

    _say("sweep R-MAT scale 18 ef 16 A*A, FP64, rounds, sampled rows")
    ac, a = _inputs("rmat", 18, 16)
    deg = np.diff(a.ptr)
    rowflop = np.bincount(np.repeat(np.arange(a.nrows), deg), weights=deg[a.idx].astype(np.float64),
                          minlength=a.nrows)
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([np.argsort(rowflop)[-16:], rng.integers(0, a.nrows, 64)]))
    ref = oracle.spgemm_rows(ac, a, rows, nthreads=len(os.sched_getaffinity(0)))
    A, B = pb.DeviceCsx.from_host(ac), pb.DeviceCsx.from_host(a)
    tune = {"round_tuples": 1 << 32}
    sym = torch.empty(pb.spgemm_symbolic(A, B, "f64", tune), dtype=torch.uint8, device="cuda")
    plan = pb.spgemm_symbolic(A, B, "f64", tune, sym_ws=sym)
    rb, fl = pb.spgemm_plan_rounds(plan)
    assert len(fl) > 1 and rb[0] == 0 and rb[-1] == a.nrows
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    maxrows = max(rb[i + 1] - rb[i] for i in range(len(fl)))
    rp = torch.empty(maxrows + 1, dtype=torch.int64, device="cuda")
    ci = torch.empty(max(fl), dtype=torch.int32, device="cuda")
    cv = torch.empty(max(fl), dtype=torch.float64, device="cuda")
    seen = 0
    for r in range(len(fl)):
        nnz = pb.spgemm_numeric_round(plan, A, B, r, ws, rp, ci, cv)
        nrows = rb[r + 1] - rb[r]
        p = rp[: nrows + 1]
        assert int(p[0]) == 0 and int(p[-1]) == nnz <= fl[r] and bool(torch.all(p[1:] >= p[:-1]))
        _sorted_rows_on_device(torch, p, ci, nrows)
        sel = rows[(rows >= rb[r]) & (rows < rb[r + 1])]
        if sel.size:
            h = p.cpu().numpy()
            idx = np.searchsorted(rows, sel)

            def get_row(row, base=rb[r], h=h):
                return ci[h[row - base]:h[row - base + 1]].cpu().numpy(), cv[h[row - base]:h[row - base + 1]].cpu().numpy()

            sub = {"ptr": np.concatenate([[0], np.cumsum(ref["ptr"][idx + 1] - ref["ptr"][idx])])}
            for key in ("idx", "val", "absval"):
                sub[key] = np.concatenate([ref[key][ref["ptr"][i]:ref["ptr"][i + 1]] for i in idx])
            _check_rows(sel, sub, get_row, "f64")
            seen += sel.size
        _say(f"round {r + 1}/{len(fl)} ok")
    assert seen == rows.size
    plan.close()
