"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Structure (row pointers and column indices) must match bit for bit.  Values
are compared against N = |A||B| of each entry (for non-negative inputs N is
the value itself, so this is the relative error): FP64 within 1e-12, FP32
tuples with compensated merge within 1e-6.
"""
import os
import sys

import numpy as np
import pytest

import oracle
from workloads import Csx, csc_to_csr, er_problem, identity, random_sparse

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32c": 1e-6}


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pb():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_11302_amd as pbm

    pbm.load()
    return pbm


def _run(pb, a: Csx, b: Csx, precision="f64", tune=None):
    A = pb.DeviceCsx.from_host(a)
    B = pb.DeviceCsx.from_host(b)
    c = pb.spgemm(A, B, precision=precision, tune=tune)
    return c.to_host()


def _compare(got: dict, ref: dict, precision: str, exact_values=False):
    assert np.array_equal(got["rowptr"], ref["rowptr"]), "row pointers differ"
    assert np.array_equal(got["colidx"], ref["colidx"]), "column indices differ"
    gv = got["val"].astype(np.float64)
    if exact_values:
        assert np.array_equal(gv, ref["val"])
        return 0.0
    err = np.abs(gv - ref["val"])
    bound = TOL[precision] * ref["absval"]
    bad = err > bound
    worst = float(np.max(np.where(ref["absval"] > 0, err / np.where(ref["absval"] > 0, ref["absval"], 1), err))) if err.size else 0.0
    assert not np.any(bad), f"{int(bad.sum())} values beyond {TOL[precision]} x N; worst ratio {worst:.3e}"
    return worst


def _check_invariants(got: dict, flop: int):
    rp, ci = got["rowptr"], got["colidx"]
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == len(ci)
    assert len(ci) <= flop
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    key = rows.astype(np.int64) * (int(ci.max()) + 1 if len(ci) else 1) + ci
    assert np.all(np.diff(key) > 0), "columns must strictly increase within rows"


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_er_4096_d4_square(pb, precision):
    _say(f"ER n=4096 d=4 A*A {precision}")
    a, b = er_problem(4096, 4, 1, None)
    ref = oracle.spgemm(a, b)
    got = _run(pb, a, b, precision)
    _compare(got, ref, precision)
    _check_invariants(got, ref["flop"])


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_er_signed_several_tiles(pb, precision):
    _say(f"ER n=60000 d=8 signed {precision}")
    a, b = er_problem(60000, 8, 5, 6, values="signed")
    ref = oracle.spgemm(a, b)
    got = _run(pb, a, b, precision)
    _compare(got, ref, precision)


@pytest.mark.parametrize("tile", [256, 1000, 2048, 4096])
@pytest.mark.parametrize("chunk", [512, 2048])
def test_tiles_and_chunks(pb, tile, chunk):
    _say(f"ER n=20011 d=6 tile={tile} chunk={chunk}")
    a, b = er_problem(20011, 6, 7, 8)
    ref = oracle.spgemm(a, b)
    got = _run(pb, a, b, "f64", tune={"tile_tuples": tile, "expand_chunk": chunk})
    _compare(got, ref, "f64")


def test_rectangular_with_dense_and_empty_lines(pb):
    _say("rectangular 3000x700x2500 with dense/empty rows and columns")
    a = random_sparse(3000, 700, 0.002, 11, "csc", values="signed", dense_rows=(17,), empty_cols=(0, 5, 699))
    b = random_sparse(700, 2500, 0.001, 12, "csr", values="signed", dense_cols=(3,), empty_rows=(2, 600))
    ref = oracle.spgemm(a, b)
    got = _run(pb, a, b, "f64")
    _compare(got, ref, "f64")


def test_isolated_big_rows_small_tile(pb):
    # rows whose flop exceeds tile/2 become single-row bins
    _say("isolated big rows with tile=512")
    a = random_sparse(900, 400, 0.01, 21, "csc", dense_rows=(5, 6, 400, 899))
    b = random_sparse(400, 700, 0.0015, 22, "csr")
    ref = oracle.spgemm(a, b)
    got = _run(pb, a, b, "f64", tune={"tile_tuples": 512})
    _compare(got, ref, "f64")


def test_integer_values_bit_exact(pb):
    _say("integer-valued inputs, exact sums")
    a = random_sparse(2000, 1500, 0.004, 31, "csc", values="int")
    b = random_sparse(1500, 1800, 0.004, 32, "csr", values="int")
    ref = oracle.spgemm(a, b)
    got = _run(pb, a, b, "f64")
    _compare(got, ref, "f64", exact_values=True)
    got32 = _run(pb, a, b, "f32c")
    _compare(got32, ref, "f32c", exact_values=True)  # small integers are exact in float too


def test_identity_products(pb):
    _say("A*I and I*B")
    a = random_sparse(5000, 3000, 0.002, 41, "csc", values="signed")
    got = _run(pb, a, identity(3000, "csr"), "f64")
    ar = csc_to_csr(a)
    assert np.array_equal(got["rowptr"], ar.ptr) and np.array_equal(got["colidx"], ar.idx)
    assert np.array_equal(got["val"], ar.val)
    b = random_sparse(3000, 4000, 0.002, 42, "csr", values="signed")
    got = _run(pb, identity(3000, "csc"), b, "f64")
    assert np.array_equal(got["rowptr"], b.ptr) and np.array_equal(got["colidx"], b.idx)
    assert np.array_equal(got["val"], b.val)


def test_empty_and_degenerate(pb):
    _say("empty / degenerate shapes")
    for (m, k, n, dens) in [(100, 50, 80, 0.0), (1, 1, 1, 1.0), (64, 1, 64, 0.5), (300, 200, 1, 0.05), (0, 10, 10, 0.1), (10, 0, 10, 0.1)]:
        a = random_sparse(m, k, dens, 51, "csc") if m and k else Csx(m, k, np.zeros(k + 1, np.int64), np.zeros(0, np.int32), np.zeros(0), "csc")
        b = random_sparse(k, n, dens, 52, "csr") if k and n else Csx(k, n, np.zeros(k + 1, np.int64), np.zeros(0, np.int32), np.zeros(0), "csr")
        ref = oracle.spgemm(a, b) if m else dict(rowptr=np.zeros(1, np.int64), colidx=np.zeros(0, np.int32), val=np.zeros(0), absval=np.zeros(0))
        got = _run(pb, a, b, "f64")
        _compare(got, ref, "f64")


def test_cancellation_stays_stored(pb):
    _say("exact cancellation")
    # A = [[1, 1]], B = [[1], [-1]]
    a = Csx(1, 2, np.array([0, 1, 2], np.int64), np.array([0, 0], np.int32), np.array([1.0, 1.0]), "csc")
    b = Csx(2, 1, np.array([0, 1, 2], np.int64), np.array([0, 0], np.int32), np.array([1.0, -1.0]), "csr")
    got = _run(pb, a, b, "f64")
    assert list(got["rowptr"]) == [0, 1] and list(got["colidx"]) == [0] and got["val"][0] == 0.0


def test_tile_invariance(pb):
    _say("structure independent of tile / chunk")
    a, b = er_problem(30000, 7, 61, 62, values="signed")
    base = _run(pb, a, b, "f64")
    for tune in ({"tile_tuples": 300}, {"tile_tuples": 2048, "expand_chunk": 2048}):
        got = _run(pb, a, b, "f64", tune=tune)
        assert np.array_equal(got["rowptr"], base["rowptr"]) and np.array_equal(got["colidx"], base["colidx"])
        assert np.allclose(got["val"], base["val"], rtol=0, atol=1e-12)


def test_row_wider_than_tile(pb):
    """A row with more tuples than the tile goes through the column-window
    path (n = 400 fits one window, so the window is summed densely)."""
    _say("row with more tuples than the tile")
    a = random_sparse(200, 300, 0.01, 71, "csc", dense_rows=(3,))
    b = random_sparse(300, 400, 0.05, 72, "csr")
    got = _run(pb, a, b, "f64", tune={"tile_tuples": 256})
    _compare(got, oracle.spgemm(a, b), "f64")


def test_capacity_error_reports_size(pb):
    import torch

    _say("capacity too small")
    a, b = er_problem(3000, 4, 81, 82)
    A = pb.DeviceCsx.from_host(a)
    B = pb.DeviceCsx.from_host(b)
    nsym = pb.spgemm_symbolic(A, B)
    plan = pb.spgemm_symbolic(A, B, sym_ws=torch.empty(nsym, dtype=torch.uint8, device="cuda"))
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    rowptr = torch.empty(a.nrows + 1, dtype=torch.int64, device="cuda")
    colidx = torch.empty(100, dtype=torch.int32, device="cuda")
    val = torch.empty(100, dtype=torch.float64, device="cuda")
    with pytest.raises(pb.PbError) as ei:
        pb.spgemm_numeric(plan, A, B, ws, rowptr, colidx, val)
    assert ei.value.name == "PB_ERR_CAPACITY"
    ref = oracle.spgemm(a, b)
    assert int(rowptr[-1].item()) == len(ref["colidx"])


@pytest.fixture(scope="module")
def er_2e20():
    """The benchmark workload and all of its C from the oracle (in CSR,
    computed row by row through (AB)^T = B^T A^T)."""
    import os

    a, b = er_problem(1 << 20, 16, 2, 3)
    _say("ER n=2^20 d=16: oracle over all rows")
    ref = oracle.spgemm_rows(a, b, None, nthreads=len(os.sched_getaffinity(0)))
    return a, b, ref


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_er_2e20_d16_full_size_whole_c(pb, er_2e20, precision):
    """The benchmark workload at full size, every entry of C against the
    oracle: row pointers and columns bit-exact, values within the tolerance
    of N = |A||B| (compared on the device)."""
    import torch

    a, b, ref = er_2e20
    _say(f"ER n=2^20 d=16 A*B whole C {precision}")
    A = pb.DeviceCsx.from_host(a)
    B = pb.DeviceCsx.from_host(b)
    c = pb.spgemm(A, B, precision=precision)
    assert c.nnz <= 16 * 16 * (1 << 20)
    assert torch.equal(c.rowptr, torch.from_numpy(ref["ptr"]).cuda()), "row pointers differ"
    assert torch.equal(c.colidx, torch.from_numpy(ref["idx"]).cuda()), "column indices differ"
    rv = torch.from_numpy(ref["val"]).cuda()
    err = (c.val.double() - rv).abs()
    del rv
    bound = torch.from_numpy(ref["absval"]).cuda().mul_(TOL[precision])
    nbad = int((err > bound).sum().item())
    worst = float((err / bound.clamp_min(1e-300)).max().item()) * TOL[precision]
    _say(f"{precision}: nnz(C) {c.nnz}, worst |d|/N {worst:.3e}")
    assert nbad == 0, f"{nbad} values beyond {TOL[precision]} x N (worst {worst:.3e})"


@pytest.mark.parametrize("tile", [1500, 2048])
def test_full_bins_repeated(pb, tile):
    """Bins filled close to the tile, run several times: per-row entry
    counts must be exact every time (a count that depended on the timing of
    the LDS hash-set inserts once lost whole per-wave row segments here)."""
    _say(f"ER 12000 d=6, tile {tile}, 4 runs")
    a, b = er_problem(12000, 6, 43, 44, values="signed")
    ref = oracle.spgemm(a, b)
    for _ in range(4):
        _compare(_run(pb, a, b, "f64", tune={"tile_tuples": tile}), ref, "f64")


@pytest.mark.parametrize("align", [1, 4, 8])
def test_run_alignment(pb, align):
    """Runs padded to 1, 4 or 8 slots (padding carries the sentinel key):
    C is the same; B's rows have uneven lengths, so runs end mid-sector."""
    import torch

    _say(f"ER 30011 d=16 run_align={align}")
    a, b = er_problem(30011, 16, 21, 22, values="signed")
    ref = oracle.spgemm(a, b)
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    for prec in ("f64", "f32c"):
        got = pb.spgemm(A, B, precision=prec, tune={"run_align": align}).to_host()
        _compare(got, ref, prec)
    nsym = pb.spgemm_symbolic(A, B, "f64", {"run_align": align})
    plan = pb.spgemm_symbolic(A, B, "f64", {"run_align": align},
                              sym_ws=torch.empty(nsym, dtype=torch.uint8, device="cuda"))
    info = plan.info()
    assert info["run_align"] == align and info["flop"] == ref["flop"]
    nb = np.diff(b.ptr)
    na = np.diff(a.ptr)
    assert info["slots"] == int(np.sum(na * ((nb + align - 1) // align * align)))
    plan.close()



def _plan_info(pb, A, B, precision, tune):
    import torch

    nsym = pb.spgemm_symbolic(A, B, precision, tune)
    plan = pb.spgemm_symbolic(A, B, precision, tune, sym_ws=torch.empty(nsym, dtype=torch.uint8, device="cuda"))
    info = plan.info()
    plan.close()
    return info


@pytest.mark.parametrize("row_count", [1, 2])
def test_row_count_modes(pb, row_count):
    """Per-row flop and run offsets by device atomics (1) or by row buckets
    (2): C is the same, and so are the plan's slots, bins and row maxima.
    The inputs span several 4096-row buckets, dense rows, empty rows and
    columns, and columns so sparse that a range of entries covers tens of
    thousands of columns."""
    cases = [er_problem(30011, 16, 21, 22, values="signed"),
             (random_sparse(9000, 700, 0.002, 11, "csc", values="signed", dense_rows=(17, 8999),
                            empty_cols=(0, 5, 699)),
              random_sparse(700, 2500, 0.001, 12, "csr", values="signed", dense_cols=(3,), empty_rows=(2, 600))),
             # about 0.2 entries per column of A: each range of entries spans
             # more columns than the LDS column table holds
             (random_sparse(9000, 100000, 2e-5, 13, "csc", values="signed"),
              random_sparse(100000, 3000, 0.003, 14, "csr", values="signed"))]
    for i, (a, b) in enumerate(cases):
        _say(f"row_count={row_count} case {i}")
        ref = oracle.spgemm(a, b)
        A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
        for prec in ("f64", "f32c"):
            _compare(pb.spgemm(A, B, precision=prec, tune={"row_count": row_count}).to_host(), ref, prec)
        info = _plan_info(pb, A, B, "f64", {"row_count": row_count})
        other = _plan_info(pb, A, B, "f64", {"row_count": 3 - row_count})
        assert info["row_count"] == row_count and other["row_count"] == 3 - row_count
        for key in ("flop", "slots", "nbins", "max_bin_tuples", "max_row_flop"):
            assert info[key] == other[key], key
    # auto picks row buckets
    assert _plan_info(pb, A, B, "f64", None)["row_count"] == 2


def test_row_bucket_run_wider_than_field(pb):
    """A row of B with more than 2^20 entries: its runs' slot count does not
    fit the bucket records' 20-bit field and is looked up from B's row
    pointers instead.  The three rows of C it reaches are far wider than the
    tile (column windows, dense accumulation)."""
    n = (1 << 20) + 5
    rng = np.random.default_rng(31)
    # B: row 0 holds every column but 0 and 7; row 1 holds 10; row 2 is empty
    r0 = np.setdiff1d(np.arange(n, dtype=np.int32), np.array([0, 7], dtype=np.int32))
    r1 = np.sort(rng.choice(n, 10, replace=False)).astype(np.int32)
    bptr = np.array([0, r0.size, r0.size + r1.size, r0.size + r1.size], dtype=np.int64)
    b = Csx(3, n, bptr, np.concatenate([r0, r1]), rng.uniform(0, 1, r0.size + r1.size), "csr")
    # A: column 0 has 3 entries in two row buckets, column 1 has 40 (a long
    # column), column 2 has 5 (its B row is empty)
    m = 5000
    c0 = np.array([5, 4100, 4999], dtype=np.int32)
    c1 = np.sort(rng.choice(m, 40, replace=False)).astype(np.int32)
    c2 = np.sort(rng.choice(m, 5, replace=False)).astype(np.int32)
    aptr = np.array([0, 3, 43, 48], dtype=np.int64)
    a = Csx(m, 3, aptr, np.concatenate([c0, c1, c2]), rng.uniform(0, 1, 48), "csc")
    ref = oracle.spgemm(a, b)
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    for prec in ("f64", "f32c"):
        _say(f"B row of 2^20 entries, row buckets, {prec}")
        got = pb.spgemm(A, B, precision=prec, tune={"row_count": 2}).to_host()
        _compare(got, ref, prec)
    info = _plan_info(pb, A, B, "f64", {"row_count": 2})
    atom = _plan_info(pb, A, B, "f64", {"row_count": 1})
    assert info["row_count"] == 2 and info["slots"] == atom["slots"] and info["max_row_flop"] == atom["max_row_flop"]


@pytest.mark.parametrize("run", [30, 50])
def test_sort_crowded_buckets(pb, run):
    """Bins whose keys spread over 2^20 columns except one B row of `run`
    consecutive columns: every row of C that reaches it puts `run` keys in
    one sort bucket.  30 keys take the per-bucket ranking fallback (more than
    a thread sorts in registers), 50 the radix-sort path."""
    _say(f"crowded buckets, run of {run}")
    rng = np.random.default_rng(run)
    n, kdim, m, d = 1 << 20, 8192, 8192, 8
    rows = []
    for k in range(kdim):
        if k % 512 == 7:
            rows.append(np.arange(1000, 1000 + run, dtype=np.int32))
        else:
            rows.append(np.sort(rng.choice(n, d, replace=False)).astype(np.int32))
    bptr = np.concatenate([[0], np.cumsum([r.size for r in rows])]).astype(np.int64)
    b = Csx(kdim, n, bptr, np.concatenate(rows), rng.uniform(0, 1, int(bptr[-1])), "csr")
    cols = [np.sort(rng.choice(m, d, replace=False)).astype(np.int32) for _ in range(kdim)]
    aptr = np.concatenate([[0], np.cumsum([c.size for c in cols])]).astype(np.int64)
    a = Csx(m, kdim, aptr, np.concatenate(cols), rng.uniform(0, 1, int(aptr[-1])), "csc")
    ref = oracle.spgemm(a, b)
    for prec in ("f64", "f32c"):
        _compare(_run(pb, a, b, prec), ref, prec)


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_sort_heavy_repeats(pb, precision):
    """Bins whose tuples repeat each key about 6 times: equal keys are first
    summed in an LDS hash table and only the distinct keys are sorted (the
    path taken when at most half of a bin's slots hold distinct keys; the
    count comes from C's row pointers).  Also with smaller tiles."""
    _say(f"heavy repeats {precision}")
    a = random_sparse(3000, 60, 0.25, 51, "csc", values="signed")
    b = random_sparse(60, 48, 0.4, 52, "csr", values="signed")
    ref = oracle.spgemm(a, b)
    assert ref["flop"] >= 4 * len(ref["colidx"])
    for tune in (None, {"tile_tuples": 2048}, {"tile_tuples": 1024}):
        _compare(_run(pb, a, b, precision, tune=tune), ref, precision)


def _one_column_pattern(m, k, n, a_rows_per_col, b_cols_per_row, seed):
    """A (m x k, CSC) with the given rows in each column and B (k x n, CSR)
    with the given columns in each row, values U(0,1)."""
    rng = np.random.default_rng(seed)
    aptr = np.concatenate([[0], np.cumsum([len(r) for r in a_rows_per_col])]).astype(np.int64)
    aidx = np.concatenate([np.asarray(r, np.int32) for r in a_rows_per_col])
    bptr = np.concatenate([[0], np.cumsum([len(c) for c in b_cols_per_row])]).astype(np.int64)
    bidx = np.concatenate([np.asarray(c, np.int32) for c in b_cols_per_row])
    a = Csx(m, k, aptr, aidx, rng.random(aidx.size), "csc")
    b = Csx(k, n, bptr, bidx, rng.random(bidx.size), "csr")
    return a, b


@pytest.mark.parametrize("case", ["t2048_n2e24", "t4096_n2e21"])
def test_last_row_of_full_bin_at_last_column(pb, case):
    """A bin of normal rows holds at most 2^rowbits - 1 rows, so the key of
    its last row at column n-1 (n a power of two) is never the all-ones
    padding sentinel.  Shapes where the bin cut once reached 2^rowbits rows:
    a row of 256 tuples then 474 empty rows (tile 2048, n = 2^24: row 475
    was row 255 of its bin), and one tuple in rows 0 and 4094 only (tile
    4096, n = 2^21: row 4094 was row 2047 of its bin)."""
    _say(f"last row of a full bin at column n-1: {case}")
    if case == "t2048_n2e24":
        n = 1 << 24
        a, b = _one_column_pattern(576, 2, n, [[0], [475]],
                                   [np.arange(256) * 65536 + 7, [n - 1]], 5)
        tile = 2048
    else:
        n = 1 << 21
        a, b = _one_column_pattern(4200, 1, n, [[0, 4094]], [[n - 1]], 6)
        tile = 4096
    ref = oracle.spgemm(a, b)
    for precision in ("f64", "f32c"):
        got = _run(pb, a, b, precision, tune={"tile_tuples": tile})
        _compare(got, ref, precision)


@pytest.mark.parametrize("case", ["er", "empty_rows", "big_rows"])
def test_bin_cut_matches_rule(pb, case):
    """The device's bin count and largest bin equal the bin-cut rule
    restated on the host (tests/test_bin_cut.py) over the rows' tuple
    counts (run alignment 1, so a row's slots are its multiplications)."""
    from test_bin_cut import bin_starts

    _say(f"bin cut vs host rule: {case}")
    tile = 1024
    if case == "er":
        a, b = er_problem(30000, 7, 61, 62)
    elif case == "empty_rows":
        a, b = _one_column_pattern(9000, 2, 1 << 20, [[0, 4000], [8999]], [np.arange(300) * 17, [5, 9, 1 << 19]], 3)
    else:
        a = random_sparse(900, 400, 0.01, 21, "csc", dense_rows=(5, 6, 400, 899))
        b = random_sparse(400, 700, 0.0015, 22, "csr")
    nnzb = np.diff(b.ptr)
    rowflop = np.bincount(a.idx, weights=np.repeat(nnzb, np.diff(a.ptr)), minlength=a.nrows).astype(np.int64)
    cb = int(b.ncols - 1).bit_length() if b.ncols > 1 else 0
    starts = bin_starts(rowflop, tile, 32 - cb)
    R = np.concatenate([[0], np.cumsum(rowflop)])
    sizes = R[np.concatenate([starts[1:], [a.nrows]])] - R[starts]
    info = _plan_info(pb, pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b), "f64",
                      {"tile_tuples": tile, "run_align": 1})
    assert info["nbins"] == starts.size
    assert info["max_bin_tuples"] == int(sizes.max())
    assert info["max_row_flop"] == int(rowflop.max())


@pytest.mark.parametrize("precision", ["f64", "f32c"])
@pytest.mark.parametrize("n", [(1 << 21) + 1, (1 << 23) + (1 << 20)])
def test_rows_beyond_direct_scan_limit(pb, precision, n):
    """Scans of more than 1024 tiles of 2048 elements (the limit up to which
    each tile combines the earlier tiles' totals itself): 1025 tiles, the
    last holding one row, and 4608 tiles (three chunks of the one-workgroup
    pass that turns the totals into prefixes).  The column-flop scan, the
    row scan and the bin cut (a non-commutative scan) take that path.  Whole
    C against the oracle."""
    _say(f"ER n={n} d=2 A*B ({precision})")
    a, b = er_problem(n, 2, 71, 72)
    got = _run(pb, a, b, precision)
    ref = oracle.spgemm(a, b, nthreads=len(os.sched_getaffinity(0)))
    _compare(got, ref, precision)
