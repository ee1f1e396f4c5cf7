"""GPU tests of the fixed summation order (tune["deterministic"] = 1).

With it, every entry of C is summed one tuple at a time in ascending order
of the inner index k (the runs of a row sit in column order of A, the bin
sort is stable), which is exactly the order of the oracle's sorted-
accumulator column product (Section 2.2 formulation; the oracle sums each
C(i,j) left to right over ascending k in double).  So in FP64 the structure
AND the values must equal the oracle's bit for bit, and in both precisions
repeated calls, other tiles, run alignments, rounds and batches must give
the same bits."""
import os
import sys

import numpy as np
import pytest

import oracle
from workloads import Csx, amg_problem, er_problem, random_sparse

pytestmark = pytest.mark.gpu
DET = {"deterministic": 1}


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


def _bits(x):
    x = np.ascontiguousarray(x)
    return x.view(np.uint64) if x.dtype == np.float64 else x.view(np.uint32)


def _same(got, ref, what):
    assert np.array_equal(got["rowptr"], ref["rowptr"]), f"{what}: row pointers"
    assert np.array_equal(got["colidx"], ref["colidx"]), f"{what}: columns"
    g, r = _bits(got["val"]), _bits(ref["val"])
    bad = np.flatnonzero(g != r)
    assert bad.size == 0, f"{what}: {bad.size} values differ in their bits (first at {bad[:3]})"


def _run(pb, a, b, precision="f64", **tune):
    t = dict(DET)
    t.update(tune)
    return pb.spgemm(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b), precision=precision, tune=t).to_host()


def _cases():
    # C = A*A on the small Erdos-Renyi workload (n = 4096, 4 entries per column)
    a, b = er_problem(4096, 4, 1, None)  # seed_b None: B is A itself, in CSR
    yield "er 4096 d4 A*A", a, b, {}
    a, b = er_problem(60000, 8, 31, 32, values="signed")
    yield "er 60000 d8", a, b, {}
    yield "er 60000 d8 tile 512", a, b, {"tile_tuples": 512}
    # repeated keys: many products land on one entry of C
    a, b = er_problem(3000, 24, 41, 42, values="signed")
    yield "er 3000 d24 (repeats)", a, b, {}
    yield "rectangular with empty lines and a dense column of B", (
        random_sparse(3000, 700, 0.002, 11, "csc", values="signed", empty_rows=(17,), empty_cols=(0, 5, 699))), (
        random_sparse(700, 2500, 0.001, 12, "csr", values="signed", dense_cols=(3,), empty_rows=(2, 600))), {}


@pytest.mark.parametrize("align", [0, 1, 8])
def test_fp64_bits_equal_oracle(pb, align):
    for what, a, b, tune in _cases():
        _say(f"{what}: align {align}")
        got = _run(pb, a, b, run_align=align, **tune)
        _same(got, oracle.spgemm(a, b), what)


def test_amg_chain_bits_equal_oracle(pb):
    """T = A*P and Ac = R*T (R = P^T) on the 16^3 Laplacian: the whole chain
    is bit-equal to the oracle's chain."""
    _say("amg 16^3 chain")
    A, P = amg_problem(16)
    a_csc = Csx(A.nrows, A.ncols, A.ptr, A.idx, A.val, "csc")  # symmetric
    t_ref = oracle.spgemm(a_csc, P)
    t = _run(pb, a_csc, P)
    _same(t, t_ref, "T = A*P")
    r_csc = Csx(P.ncols, P.nrows, P.ptr, P.idx, P.val, "csc")
    t_csr = Csx(A.nrows, P.ncols, t["rowptr"], t["colidx"], t["val"], "csr")
    _same(_run(pb, r_csc, t_csr), oracle.spgemm(r_csc, t_csr), "Ac = R*T")


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_repeatable_and_tile_invariant(pb, precision):
    a, b = er_problem(60000, 8, 51, 52, values="signed")
    _say(f"repeat {precision}")
    first = _run(pb, a, b, precision)
    for rep in range(2):
        _same(_run(pb, a, b, precision), first, f"repeat {rep}")
    for tile in (256, 1024, 4096):
        _say(f"tile {tile} {precision}")
        _same(_run(pb, a, b, precision, tile_tuples=tile), first, f"tile {tile}")
    _say(f"expand chunk 256 {precision}")
    _same(_run(pb, a, b, precision, expand_chunk=256), first, "expand chunk 256")


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_rounds_match_one_pass(pb, precision):
    a, b = er_problem(20000, 10, 61, 62, values="signed")
    _say(f"rounds {precision}")
    one = _run(pb, a, b, precision)
    rounds = _run(pb, a, b, precision, round_tuples=40000)
    _same(rounds, one, "rounds")
    if precision == "f64":
        _same(one, oracle.spgemm(a, b), "oracle")


def test_batched_bits_equal_oracle(pb):
    probs = [er_problem(int(n), int(d), 700 + i, 800 + i, values="signed")
             for i, (n, d) in enumerate([(3000, 5), (50, 2), (7000, 9), (1, 1), (2500, 3), (4096, 16)])]
    pairs = [(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)) for a, b in probs]
    for tile in (1024, 4096):
        _say(f"batch of {len(probs)}, tile {tile}")
        outs = pb.spgemm_batch(pairs, precision="f64", tune={"deterministic": 1, "tile_tuples": tile})
        for i, ((a, b), c) in enumerate(zip(probs, outs)):
            _same(c.to_host(), oracle.spgemm(a, b), f"problem {i}")
    _say("batch f32c against single products")
    outs = pb.spgemm_batch(pairs, precision="f32c", tune=DET)
    for i, ((a, b), c) in enumerate(zip(probs, outs)):
        _same(c.to_host(), _run(pb, a, b, "f32c", tile_tuples=4096), f"problem {i} f32c")


def test_wide_rows_refused(pb):
    """A row of C wider than the tile has no fixed order here: the symbolic
    step refuses the plan (the default mode takes it)."""
    from paper_2002_11302_amd._binding import PbError

    _say("wide row refused")
    a = random_sparse(900, 400, 0.01, 21, "csc", dense_rows=(5,))
    b = random_sparse(400, 700, 0.02, 22, "csr")
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    with pytest.raises(PbError) as ei:
        pb.spgemm(A, B, tune={"deterministic": 1, "tile_tuples": 256})
    assert ei.value.name == "PB_ERR_UNSUPPORTED"
    pb.spgemm(A, B, tune={"tile_tuples": 256})


def test_headline_product_bits_equal_oracle(pb):
    """The benchmark's product (ER n=2^20, d=16, C = A*B: 2.7e8
    multiplications), all of C: in the fixed order its FP64 values are the
    oracle's bit for bit."""
    _say("ER 2^20 d16 A*B, fixed order, all of C")
    a, b = er_problem(1 << 20, 16, 2, 3)
    got = _run(pb, a, b)
    _same(got, oracle.spgemm(a, b, nthreads=len(os.sched_getaffinity(0))), "ER 2^20 d16")


def test_amg_128_chain_bits_equal_oracle(pb):
    """The AMG chain of the benchmark (7-point Laplacian 128^3): T = A*P and
    Ac = R*T, both bit-equal to the oracle's chain in the fixed order."""
    _say("amg 128^3 chain, fixed order")
    A, P = amg_problem(128)
    nth = len(os.sched_getaffinity(0))
    a_csc = Csx(A.nrows, A.ncols, A.ptr, A.idx, A.val, "csc")
    t_ref = oracle.spgemm(a_csc, P, nthreads=nth)
    t = _run(pb, a_csc, P)
    _same(t, t_ref, "T = A*P")
    r_csc = Csx(P.ncols, P.nrows, P.ptr, P.idx, P.val, "csc")
    t_csr = Csx(A.nrows, P.ncols, t["rowptr"], t["colidx"], t["val"], "csr")
    _same(_run(pb, r_csc, t_csr), oracle.spgemm(r_csc, t_csr, nthreads=nth), "Ac = R*T")
