"""GPU parity for batched products C_i = A_i * B_i (one block-diagonal
launch set for the whole batch), including a HIP-graph capture."""
import sys

import numpy as np
import pytest

import oracle
from workloads import Csx, batched_er_sizes, er_problem, random_sparse

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


def _empty(m, k, fmt):
    nmaj = k if fmt == "csc" else m
    return Csx(m, k, np.zeros(nmaj + 1, np.int64), np.zeros(0, np.int32), np.zeros(0), fmt)


def _uneven_batch(seed=5):
    probs = []
    rng = np.random.default_rng(seed)
    for i in range(10):
        n = int(rng.integers(50, 3000))
        d = int(rng.integers(1, 9))
        probs.append(er_problem(n, d, 100 + i, 200 + i, values="signed"))
    probs.append((random_sparse(300, 200, 0.02, 7, "csc"), random_sparse(200, 250, 0.02, 8, "csr")))
    probs.append((_empty(0, 40, "csc"), random_sparse(40, 30, 0.1, 9, "csr")))    # no rows
    probs.append((_empty(25, 0, "csc"), _empty(0, 35, "csr")))                      # inner dimension 0
    probs.append((random_sparse(64, 50, 0.0, 10, "csc"), random_sparse(50, 64, 0.1, 11, "csr")))  # empty A
    return probs


def _check(got: dict, ref: dict, precision: str):
    assert np.array_equal(got["rowptr"], ref["rowptr"])
    assert np.array_equal(got["colidx"], ref["colidx"])
    err = np.abs(got["val"].astype(np.float64) - ref["val"])
    assert np.all(err <= TOL[precision] * ref["absval"])


def _ref(a, b):
    if a.nrows == 0:
        return dict(rowptr=np.zeros(1, np.int64), colidx=np.zeros(0, np.int32), val=np.zeros(0), absval=np.zeros(0))
    return oracle.spgemm(a, b)


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_uneven_batch(pb, precision):
    _say(f"uneven batch of 14 {precision}")
    probs = _uneven_batch()
    pairs = [(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)) for a, b in probs]
    outs = pb.spgemm_batch(pairs, precision=precision)
    for (a, b), c in zip(probs, outs):
        _check(c.to_host(), _ref(a, b), precision)


def test_batch_of_one_and_single_path_agree(pb):
    _say("batch of one vs single product")
    a, b = er_problem(5000, 6, 31, 32, values="signed")
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    (cb,) = pb.spgemm_batch([(A, B)])
    cs = pb.spgemm(A, B)
    gb, gs = cb.to_host(), cs.to_host()
    assert np.array_equal(gb["rowptr"], gs["rowptr"]) and np.array_equal(gb["colidx"], gs["colidx"])
    _check(gb, oracle.spgemm(a, b), "f64")


def test_batch_sizes_like_workload(pb):
    """The batched workload's size law (log-uniform n, d in 2..32), scaled
    down to n <= 2^12 so the oracle stays fast."""
    _say("log-uniform batch of 48, n <= 2^12")
    n, d = batched_er_sizes(48, seed=4, lo_log2=6, hi_log2=12)
    probs = [er_problem(int(n[i]), int(min(d[i], n[i] // 4)), 1000 + i, 2000 + i, values="signed") for i in range(48)]
    pairs = [(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)) for a, b in probs]
    for prec in ("f64", "f32c"):
        outs = pb.spgemm_batch(pairs, precision=prec, tune={"tile_tuples": 4096})
        for (a, b), c in zip(probs, outs):
            _check(c.to_host(), oracle.spgemm(a, b), prec)


def test_graph_capture_replays(pb):
    """The numeric step enqueues work only (no sync): capture it in a HIP
    graph and replay it several times, with eager work and synchronisations
    between replays; every replay must equal the eager result and the
    oracle."""
    import torch

    _say("hipGraph capture of the batched numeric step")
    probs = _uneven_batch(seed=9)[:8]
    pairs = [(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)) for a, b in probs]
    nsym = pb.spgemm_batched_symbolic(pairs)
    plan = pb.spgemm_batched_symbolic(pairs, sym_ws=torch.empty(nsym, dtype=torch.uint8, device="cuda"))
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    outs = [(torch.empty(a.nrows + 1, dtype=torch.int64, device="cuda"),
             torch.empty(max(f, 1), dtype=torch.int32, device="cuda"),
             torch.empty(max(f, 1), dtype=torch.float64, device="cuda")) for (a, _), f in zip(pairs, plan.flops)]
    nnz = pb.spgemm_batched(plan, pairs, ws, outs, sync=True)
    eager = [(rp.clone(), ci[:z].clone(), cv[:z].clone()) for (rp, ci, cv), z in zip(outs, nnz)]
    refs = [_ref(a, b) for a, b in probs]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        pb.spgemm_batched(plan, pairs, ws, outs, sync=False, stream=side)  # warm-up on the side stream
        side.synchronize()
        with torch.cuda.graph(g, stream=side):
            pb.spgemm_batched(plan, pairs, ws, outs, sync=False, stream=side)
    torch.cuda.synchronize()
    for rep in range(3):
        for rp, ci, cv in outs:  # scribble over the outputs between replays
            rp.fill_(-1)
            ci.fill_(-1)
            cv.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (rp, ci, cv), (erp, eci, ecv), z, ref in zip(outs, eager, nnz, refs):
            assert torch.equal(rp, erp), f"replay {rep}: row pointers"
            assert torch.equal(ci[:z], eci), f"replay {rep}: columns"
            assert torch.allclose(cv[:z], ecv, rtol=1e-12, atol=0), f"replay {rep}: values"
            _check(dict(rowptr=rp.cpu().numpy(), colidx=ci[:z].cpu().numpy(), val=cv[:z].cpu().numpy()), ref, "f64")
    plan.close()


def test_batch_with_wide_row_is_rejected(pb):
    """Batched products need every row of C within the tile."""
    _say("batch with a row wider than the tile")
    wide = (random_sparse(50, 300, 0.01, 91, "csc", dense_rows=(3,)), random_sparse(300, 400, 0.05, 92, "csr"))
    probs = [er_problem(500, 3, 93, 94), wide]
    pairs = [(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)) for a, b in probs]
    with pytest.raises(pb.PbError) as ei:
        pb.spgemm_batch(pairs, tune={"tile_tuples": 256})
    assert ei.value.name == "PB_ERR_UNSUPPORTED"



def _compare_device(c, ref, precision, what):
    """C (device CSR) against oracle arrays (ptr/idx/val/absval), on the device."""
    import torch

    assert torch.equal(c.rowptr, torch.from_numpy(ref["ptr"]).cuda()), f"{what}: row pointers"
    assert torch.equal(c.colidx, torch.from_numpy(ref["idx"]).cuda()), f"{what}: columns"
    err = (c.val.double() - torch.from_numpy(ref["val"]).cuda()).abs()
    bound = torch.from_numpy(ref["absval"]).cuda() * TOL[precision]
    assert bool(torch.all(err <= bound).item()), f"{what}: values beyond {TOL[precision]} x N"


def _compare_rows(c, ref, rows, precision, what):
    rp = c.rowptr.cpu().numpy()
    ci = c.colidx.cpu().numpy()
    cv = c.val.cpu().numpy().astype(np.float64)
    for s, r in enumerate(rows):
        lo, hi = rp[r], rp[r + 1]
        rlo, rhi = ref["ptr"][s], ref["ptr"][s + 1]
        assert np.array_equal(ci[lo:hi], ref["idx"][rlo:rhi]), f"{what}: row {r} structure"
        assert np.all(np.abs(cv[lo:hi] - ref["val"][rlo:rhi]) <= TOL[precision] * ref["absval"][rlo:rhi]), \
            f"{what}: row {r} values"


@pytest.mark.slow
def test_batch_512_workload_vs_oracle(pb):
    """The benchmarked batch itself (512 ER products, n_i log-uniform in
    [2^10, 2^17], d_i in 2..32, values U(-1,1), 5.9e9 multiplications), in
    the benchmark's configuration (2048-tuple bins, 1024-tuple expand
    chunks) and with 4096-tuple bins, FP64 and FP32c.  Whole C against the
    oracle for every 4th problem of the FP64 2048-tuple run and every 16th
    of the others; 8 random rows of every other problem of the FP64
    2048-tuple run; CSR invariants of every problem in every run."""
    import os

    import torch

    from workloads import batched_er_problems

    nth = len(os.sched_getaffinity(0))
    _say("batch of 512: generating")
    probs = list(batched_er_problems(512))
    pairs = [(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)) for a, b in probs]
    rng = np.random.default_rng(512)
    for precision, tile, stride in (("f64", 2048, 4), ("f32c", 2048, 16), ("f64", 4096, 16), ("f32c", 4096, 16)):
        _say(f"batch of 512: {precision}, tile {tile}")
        outs = pb.spgemm_batch(pairs, precision=precision, tune={"tile_tuples": tile, "expand_chunk": 1024})
        for i, ((a, b), c) in enumerate(zip(probs, outs)):
            what = f"{precision} tile {tile} problem {i}"
            rp = c.rowptr
            flop = int(np.dot(np.diff(a.ptr), np.diff(b.ptr)))
            assert int(rp[0]) == 0 and int(rp[-1]) == c.nnz <= flop, f"{what}: row pointer ends"
            assert bool(torch.all(rp[1:] >= rp[:-1]).item()), f"{what}: row pointers decrease"
            if i % stride == 0:
                _compare_device(c, oracle.spgemm_rows(a, b, None, nthreads=nth), precision, what)
            elif stride == 4:
                rows = np.unique(rng.integers(0, a.nrows, 8))
                _compare_rows(c, oracle.spgemm_rows(a, b, rows, nthreads=nth), rows, precision, what)
        del outs
        torch.cuda.empty_cache()


def test_back_to_back_calls_into_different_outputs(pb):
    """Two stream-ordered calls on one plan, each into its own outputs, with
    no synchronisation between them: the second call's descriptors must not
    overwrite the first's before the first has uploaded them."""
    import torch

    _say("two unsynchronised batched calls, different outputs")
    probs = _uneven_batch(seed=13)[:6]
    pairs = [(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)) for a, b in probs]
    nsym = pb.spgemm_batched_symbolic(pairs)
    plan = pb.spgemm_batched_symbolic(pairs, sym_ws=torch.empty(nsym, dtype=torch.uint8, device="cuda"))
    ws = [torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda") for _ in range(2)]

    def outputs():
        return [(torch.full((a.nrows + 1,), -1, dtype=torch.int64, device="cuda"),
                 torch.full((max(f, 1),), -1, dtype=torch.int32, device="cuda"),
                 torch.full((max(f, 1),), float("nan"), dtype=torch.float64, device="cuda"))
                for (a, _), f in zip(pairs, plan.flops)]

    o1, o2 = outputs(), outputs()
    torch.cuda.synchronize()
    pb.spgemm_batched(plan, pairs, ws[0], o1, sync=False)
    pb.spgemm_batched(plan, pairs, ws[1], o2, sync=False)
    torch.cuda.synchronize()
    for outs in (o1, o2):
        for (a, b), (rp, ci, cv) in zip(probs, outs):
            ref = _ref(a, b)
            z = int(rp[-1].item())
            _check(dict(rowptr=rp.cpu().numpy(), colidx=ci[:z].cpu().numpy(), val=cv[:z].cpu().numpy()), ref, "f64")
    plan.close()


def test_size_classes_match_oracle(pb, tmp_path):
    """A batch cut into flop size classes (each class its own block-diagonal
    batch with its own tile): every product equals the oracle, with fixed
    per-class tunings, with tunings the tuner picks (cache in a temporary
    file), and when the numeric steps of all classes are replayed from one
    HIP graph."""
    import torch

    from paper_2002_11302_amd import autotune

    probs = _uneven_batch(seed=13)
    probs.append(er_problem(20000, 16, 301, 302, values="signed"))  # the largest class
    pairs = [(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)) for a, b in probs]
    flops = [int(np.dot(np.diff(a.ptr), np.diff(b.ptr))) if a.ncols else 0 for a, b in probs]
    bounds = (1 << 14, 1 << 20)
    groups = autotune.size_classes(flops, bounds)
    assert len(groups) == 3 and sorted(sum(groups, [])) == list(range(len(probs)))
    refs = [_ref(a, b) for a, b in probs]

    def outputs(prec):
        vdt = torch.float64 if prec == "f64" else torch.float32
        return [(torch.empty(a.nrows + 1, dtype=torch.int64, device="cuda"),
                 torch.empty(max(f, 1), dtype=torch.int32, device="cuda"),
                 torch.empty(max(f, 1), dtype=vdt, device="cuda")) for (a, _), f in zip(pairs, flops)]

    def check(outs, nnz, prec, what):
        for i, ((rp, ci, cv), z, ref) in enumerate(zip(outs, nnz, refs)):
            got = dict(rowptr=rp.cpu().numpy(), colidx=ci[:z].cpu().numpy(), val=cv[:z].cpu().numpy())
            _check(got, ref, prec)

    for prec in ("f64", "f32c"):
        _say(f"size classes, fixed tunings, {prec}")
        tunes = [{"tile_tuples": 1024, "expand_chunk": 256}, {"tile_tuples": 2048, "expand_chunk": 1024},
                 {"tile_tuples": 4096, "expand_chunk": 2048}]
        cb = autotune.ClassedBatch(pairs, prec, flops, bounds=bounds, tunes=tunes)
        outs = outputs(prec)
        check(outs, cb.run(outs, sync=True), prec, "fixed")
        cb.close()
    _say("size classes, tuned, then one graph")
    cb = autotune.ClassedBatch(pairs, "f64", flops, bounds=bounds)
    outs = outputs("f64")
    chosen = cb.choose(outs, reps=1, path=str(tmp_path / "tune.json"))
    assert [c["count"] for c in chosen] == [len(g) for g in groups]
    cb.symbolic()
    nnz = cb.run(outs, sync=True)
    check(outs, nnz, "f64", "tuned")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        cb.run(outs, sync=False, stream=side)
        side.synchronize()
        with torch.cuda.graph(g, stream=side):
            cb.run(outs, sync=False, stream=side)
    torch.cuda.synchronize()
    for rep in range(2):
        for rp, ci, cv in outs:
            rp.fill_(-1)
            ci.fill_(-1)
            cv.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check(outs, nnz, "f64", f"replay {rep}")
    cb.close()
