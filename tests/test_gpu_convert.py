"""GPU parity of the two ConvertCSR modes (C's row pointers from a count
pass and a row scan before the sort, or fused into the sort by a decoupled
look-back over the bins) against the oracle, on single products, products
in rounds with rows wider than the tile, batches, and bins whose crowded
sort buckets send them through the hash pre-summation (which succeeds when
keys repeat and gives up when too many keys are distinct)."""
import sys

import numpy as np
import pytest

import oracle
from workloads import Csx, er_problem, random_sparse

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


def _compare(got, ref, precision, what):
    assert np.array_equal(got["rowptr"], ref["rowptr"]), f"{what}: row pointers"
    assert np.array_equal(got["colidx"], ref["colidx"]), f"{what}: columns"
    err = np.abs(got["val"].astype(np.float64) - ref["val"])
    assert np.all(err <= TOL[precision] * ref["absval"]), f"{what}: values"


def _pattern(m, k, n, a_rows_per_col, b_cols_per_row, seed):
    rng = np.random.default_rng(seed)
    aptr = np.concatenate([[0], np.cumsum([len(r) for r in a_rows_per_col])]).astype(np.int64)
    aidx = np.concatenate([np.asarray(r, np.int32) for r in a_rows_per_col])
    bptr = np.concatenate([[0], np.cumsum([len(c) for c in b_cols_per_row])]).astype(np.int64)
    bidx = np.concatenate([np.asarray(c, np.int32) for c in b_cols_per_row])
    return (Csx(m, k, aptr, aidx, rng.uniform(-1, 1, aidx.size), "csc"),
            Csx(k, n, bptr, bidx, rng.uniform(-1, 1, bidx.size), "csr"))


def _cases():
    yield "er 30000 d7", er_problem(30000, 7, 61, 62, values="signed"), None
    yield "rectangular with dense/empty lines", (
        random_sparse(3000, 700, 0.002, 11, "csc", values="signed", dense_rows=(17,), empty_cols=(0, 5, 699)),
        random_sparse(700, 2500, 0.001, 12, "csr", values="signed", dense_cols=(3,), empty_rows=(2, 600))), None
    # bins that are all empty rows between sparse ones
    yield "mostly empty rows", _pattern(9000, 2, 1 << 20, [[0, 4000], [8999]],
                                        [np.arange(300) * 17, [5, 9, 1 << 19]], 3), {"tile_tuples": 512}
    # crowded buckets whose keys repeat: the hash pre-summation succeeds
    rep = [np.arange(200) * 3 + 1000 for _ in range(4)]
    yield "crowded, repeated keys", _pattern(64, 4, 1 << 20, [[0, 1, 40]] * 4, rep, 4), None
    # crowded buckets of distinct keys: the hash pre-summation gives up
    yield "crowded, distinct keys", _pattern(64, 1, 1 << 20, [[0, 1]], [np.arange(1000) + 5000], 5), None
    # rounds with rows wider than the tile
    yield "rounds and wide rows", (
        random_sparse(3000, 900, 0.004, 305, "csc", values="signed", dense_rows=(7, 2999)),
        random_sparse(900, 2500, 0.004, 306, "csr", values="signed")), {"tile_tuples": 512, "round_tuples": 20000}


@pytest.mark.parametrize("convert", [1, 2])
@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_convert_modes_single(pb, convert, precision):
    for what, (a, b), tune in _cases():
        _say(f"{what}: convert {convert} {precision}")
        ref = oracle.spgemm(a, b)
        t = dict(tune or {})
        t["convert"] = convert
        got = pb.spgemm(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b), precision=precision, tune=t).to_host()
        _compare(got, ref, precision, what)


@pytest.mark.parametrize("convert", [1, 2])
def test_convert_modes_rounds_one_at_a_time(pb, convert):
    """Rounds taken one at a time: each round's row pointers start at 0."""
    import torch

    a = random_sparse(3000, 900, 0.004, 307, "csc", values="signed", dense_rows=(7, 1500))
    b = random_sparse(900, 2500, 0.004, 308, "csr", values="signed")
    ref = oracle.spgemm(a, b)
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    tune = {"tile_tuples": 512, "round_tuples": 15000, "convert": convert}
    nsym = pb.spgemm_symbolic(A, B, "f64", tune)
    plan = pb.spgemm_symbolic(A, B, "f64", tune, sym_ws=torch.empty(nsym, dtype=torch.uint8, device="cuda"))
    rb, fl = pb.spgemm_plan_rounds(plan)
    assert len(fl) > 2
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    for r in range(len(fl)):
        nrows = rb[r + 1] - rb[r]
        rp = torch.empty(nrows + 1, dtype=torch.int64, device="cuda")
        ci = torch.empty(max(fl[r], 1), dtype=torch.int32, device="cuda")
        cv = torch.empty(max(fl[r], 1), dtype=torch.float64, device="cuda")
        nnz = pb.spgemm_numeric_round(plan, A, B, r, ws, rp, ci, cv)
        lo, hi = ref["rowptr"][rb[r]], ref["rowptr"][rb[r + 1]]
        got = dict(rowptr=rp.cpu().numpy(), colidx=ci[:nnz].cpu().numpy(), val=cv[:nnz].cpu().numpy())
        sub = dict(rowptr=ref["rowptr"][rb[r]:rb[r + 1] + 1] - lo, colidx=ref["colidx"][lo:hi], val=ref["val"][lo:hi],
                   absval=ref["absval"][lo:hi])
        _compare(got, sub, "f64", f"round {r}")
    plan.close()


@pytest.mark.parametrize("convert", [1, 2])
def test_convert_modes_batched(pb, convert):
    probs = [er_problem(int(n), int(d), 400 + i, 500 + i, values="signed")
             for i, (n, d) in enumerate([(3000, 5), (50, 2), (7000, 9), (1, 1), (2500, 3)])]
    probs.insert(2, (Csx(0, 40, np.zeros(41, np.int64), np.zeros(0, np.int32), np.zeros(0), "csc"),
                     random_sparse(40, 30, 0.1, 9, "csr")))
    pairs = [(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)) for a, b in probs]
    for precision in ("f64", "f32c"):
        _say(f"batch of {len(probs)}: convert {convert} {precision}")
        outs = pb.spgemm_batch(pairs, precision=precision, tune={"convert": convert, "tile_tuples": 1024})
        for i, ((a, b), c) in enumerate(zip(probs, outs)):
            if a.nrows == 0:
                assert c.rowptr.cpu().numpy().tolist() == [0]
                continue
            _compare(c.to_host(), oracle.spgemm(a, b), precision, f"problem {i}")
