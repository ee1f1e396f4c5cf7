#!/usr/bin/env python3
"""Benchmark of the PB-SpGEMM hot path on one MI355X.

One step is the whole path for one product C = A*B: the symbolic step
(Algorithm 3's flop scan, per-row flop, bin cut; one host sync to size the
workspace) and the numeric step (expand into bins, per-bin LDS sort and
merge, CSR emission).  Inputs are resident in HBM before timing starts.

Workload (default): Erdos-Renyi A and B, n = 2^20, exactly 16 nonzeros per
column, values U[0,1) in double, C = A*B, FP64 path.

Beside the headline the default run times the other workloads of the
path, each reported under "extras": the same product with FP32 tuple values
and compensated sums (speedup and error against FP64), the AMG Galerkin
chain, the 512-product batch (against the plain path run product by
product), and R-MAT scale 20 in row-range rounds.  The CPU oracle computes
the whole headline product on the host (cpu_baseline), and its output also
checks this run's GPU results.

Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--precision f64|f32c] [--no-cpu-baseline]
                    [--quick [--extras] [--amg] [--batched] [--rmat]] [--sweep]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
PEAK_HBM_GBPS = 8000.0  # MI355X HBM3E, published
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2002_11302_amd", "csrc", "pb_kernels.h")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def model_bytes(m, k, nnz_a, nnz_b, flop, nnz_c, precision: str) -> dict:
    """Algorithmic bytes per phase (traffic model of the paper's Table 3 with
    this library's widths: int64 pointers, int32 indices, double inputs, packed
    32-bit keys; tuple = key + value, C entry = column + value)."""
    bt = 12 if precision == "f64" else 8
    bc = 12 if precision == "f64" else 8
    expand = 16 * (k + 1) + 12 * (nnz_a + nnz_b) + bt * flop
    sort_compress = bt * flop + bc * nnz_c + 8 * (m + 1)
    return {"expand": expand, "sort_compress": sort_compress, "total": expand + sort_compress,
            "paper_b16": 16 * (nnz_a + nnz_b + 2 * flop + nnz_c)}


def kernel_source_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def traffic_for(kernel_key: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None
    when absent or taken on another version of the kernels."""
    try:
        with open(TRAFFIC_FILE) as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    ent = data.get(kernel_key)
    if not ent or ent.get("kernel_source_sha256") != kernel_source_sha():
        return None
    return ent.get("bytes_per_launch")


def build_inputs(pb, torch):
    from workloads import er_problem

    t = time.time()
    a, b = er_problem(1 << 20, 16, 2, 3)
    log(f"generated ER n=2^20 d=16 in {time.time() - t:.1f}s")
    A = pb.DeviceCsx.from_host(a)
    B = pb.DeviceCsx.from_host(b)
    torch.cuda.synchronize()
    return a, b, A, B


def make_step(pb, torch, A, B, precision, tune=None):
    nsym = pb.spgemm_symbolic(A, B, precision, tune)
    sym_ws = torch.empty(nsym, dtype=torch.uint8, device="cuda")
    plan = pb.spgemm_symbolic(A, B, precision, tune, sym_ws=sym_ws)
    flop = plan.flop
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    plan.close()
    rowptr = torch.empty(A.nrows + 1, dtype=torch.int64, device="cuda")
    colidx = torch.empty(max(flop, 1), dtype=torch.int32, device="cuda")
    val = torch.empty(max(flop, 1), dtype=torch.float64 if precision == "f64" else torch.float32, device="cuda")

    def step():
        p = pb.spgemm_symbolic(A, B, precision, tune, sym_ws=sym_ws)
        pb.spgemm_numeric(p, A, B, ws, rowptr, colidx, val, sync=False)
        p.close()

    return step, flop, (rowptr, colidx, val)


def make_step_outputs(out):
    """(rowptr, colidx, val) of a make_step output trimmed to nnz(C)."""
    rp, ci, cv = out
    n = int(rp[-1].item())
    return rp, ci[:n], cv[:n]


def time_steps(torch, pb, step, steps, warmup):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    pb.spgemm_profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = pb.spgemm_profile_end()
    return (t1 - t0) / steps, prof


def copy_bandwidth(pb, torch, nbytes=4 << 30, reps=10):
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    pb.spgemm_copy(dst, src, nbytes)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        pb.spgemm_copy(dst, src, nbytes)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(a, b, torch=None, gpu_results=None):
    """The oracle on every host thread, over the whole benchmark product
    (row by row).  With gpu_results {precision: (rowptr, colidx, val)} on the
    device, the same oracle output also checks them: structure equal, and the
    largest |difference| / N with N = |A||B| per entry."""
    import oracle

    threads = len(os.sched_getaffinity(0))
    oracle.build(force=False)
    t = time.perf_counter()
    r = oracle.spgemm_rows(a, b, None, nthreads=threads)
    dt = time.perf_counter() - t
    flop = oracle.flop(a.ptr, b.ptr)
    out = {"value": round(2.0 * flop / dt / 1e9, 4), "unit": "GFLOPS", "cores": threads, "kind": "oracle",
           "sample": f"full product: all {a.nrows} rows of the ER n=2^20 d=16 A*B workload, FP64; "
                     f"{dt:.2f} s wall on {threads} host threads"}
    check = {}
    if gpu_results:
        ptr = torch.from_numpy(r["ptr"]).cuda()
        idx = torch.from_numpy(r["idx"]).cuda()
        val = torch.from_numpy(r["val"]).cuda()
        nrm = torch.from_numpy(r["absval"]).cuda()
        for prec, (rp, ci, cv) in gpu_results.items():
            same = bool(torch.equal(rp, ptr)) and bool(torch.equal(ci, idx))
            err = float(((cv.double() - val).abs() / nrm.clamp_min(1e-300)).max().item()) if same and val.numel() else None
            check[prec] = {"structure_equal": same, "max_err_over_N": err}
        del ptr, idx, val, nrm
    del r
    return out, check


def _abs_csx(pb, X):
    return pb.DeviceCsx(X.nrows, X.ncols, X.ptr, X.idx, X.val.abs())


def fp32c_error(pb, torch, A, B, signed):
    """Largest |C_f32c - C_f64| / N over all of C, where N = |A||B| per entry
    (for signed inputs computed on the GPU as the FP64 product of |A| and |B|,
    which has C's structure; for non-negative inputs N = C).  The FP64 result
    is itself held to 1e-12 N of the oracle by the parity tests.  Also the
    99.9th percentile.  Structure must be identical."""
    c64 = pb.spgemm(A, B, precision="f64")
    c32 = pb.spgemm(A, B, precision="f32c")
    assert torch.equal(c64.rowptr, c32.rowptr) and torch.equal(c64.colidx, c32.colidx), "FP32c structure differs"
    if signed:
        n = pb.spgemm(_abs_csx(pb, A), _abs_csx(pb, B), precision="f64")
        assert torch.equal(n.colidx, c64.colidx)
        nv = n.val
    else:
        nv = c64.val.abs()
    nz = nv > 0
    rel = (c32.val.double() - c64.val).abs()[nz] / nv[nz]
    out = {"max": float(rel.max().item()) if rel.numel() else 0.0,
           "p99.9": float(torch.quantile(rel[:: max(1, rel.numel() // 4_000_000)].float(), 0.999).item())
           if rel.numel() else 0.0}
    del c64, c32, rel
    torch.cuda.empty_cache()
    return out


def amg_f32c_error(pb, torch):
    """FP32c against FP64 for both products of the AMG chain (the second on
    the FP64 T), normalised by N = |A||B| of each entry."""
    from workloads import Csx, amg_problem

    A, P = amg_problem(128)
    Ad = pb.DeviceCsx.from_host(Csx(A.nrows, A.ncols, A.ptr, A.idx, A.val, "csc"))
    Pd = pb.DeviceCsx.from_host(P)
    T = pb.spgemm(Ad, Pd)
    Td = pb.DeviceCsx(T.nrows, T.ncols, T.rowptr, T.colidx, T.val)
    out = {"T=A*P": fp32c_error(pb, torch, Ad, Pd, signed=True),
           "Ac=R*T": fp32c_error(pb, torch, Pd.transpose_view(), Td, signed=True)}
    del T, Td
    torch.cuda.empty_cache()
    return out


def batched_f32c_error(pb, torch, count=512):
    """FP32c against FP64 over every product of the batch, normalised by
    N = |A_i||B_i| (both batches through the batched path)."""
    from workloads import batched_er_problems

    pairs = [(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)) for a, b in batched_er_problems(count)]
    worst = 0.0
    for lo in range(0, count, 64):  # 64 problems at a time bounds the memory
        chunk = pairs[lo:lo + 64]
        c64 = pb.spgemm_batch(chunk, precision="f64")
        c32 = pb.spgemm_batch(chunk, precision="f32c")
        nn = pb.spgemm_batch([(_abs_csx(pb, a), _abs_csx(pb, b)) for a, b in chunk], precision="f64")
        for x, y, z in zip(c64, c32, nn):
            assert torch.equal(x.colidx, y.colidx) and torch.equal(x.colidx, z.colidx), "FP32c structure differs"
            nz = z.val > 0
            if bool(nz.any().item()):
                worst = max(worst, float(((y.val.double() - x.val).abs()[nz] / z.val[nz]).max().item()))
        del c64, c32, nn
        torch.cuda.empty_cache()
    return {"max": worst}


def _batch_plan(pb, torch, pairs, prec, tune):
    nsym = pb.spgemm_batched_symbolic(pairs, prec, tune)
    sym = torch.empty(nsym, dtype=torch.uint8, device="cuda")
    plan = pb.spgemm_batched_symbolic(pairs, prec, tune, sym_ws=sym)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    return sym, plan, ws


def _outputs(torch, pairs, flops, prec):
    vdt = torch.float64 if prec == "f64" else torch.float32
    return [(torch.empty(a.nrows + 1, dtype=torch.int64, device="cuda"),
             torch.empty(max(f, 1), dtype=torch.int32, device="cuda"),
             torch.empty(max(f, 1), dtype=vdt, device="cuda")) for (a, _), f in zip(pairs, flops)]


def _graph_ms(torch, launch, steps, warmup):
    """Capture launch(stream) once in a HIP graph (after one eager run on the
    side stream) and time its replays."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        launch(side)
        side.synchronize()
        with torch.cuda.graph(g, stream=side):
            launch(side)
    torch.cuda.synchronize()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_batched(pb, torch, steps, warmup):
    """Batched ER workload: 512 products, n_i log-uniform in [2^10, 2^17],
    d_i in {2..32}, values U[-1,1).  The autotuner picks the tile (bin width)
    and the expand chunk for the batch's size class; the batch is timed as a
    whole path (symbolic + numeric) and with its numeric step captured in
    one HIP graph.  The baseline is the plain path run product by product
    with every plan, workspace and output allocated beforehand (whole path:
    symbolic + numeric per product; numeric: the 512 numeric calls captured
    in one graph), so no allocation is inside any timed region."""
    from paper_2002_11302_amd import autotune
    from workloads import batched_er_problems, batched_er_sizes

    t = time.time()
    pairs = [(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)) for a, b in batched_er_problems(512)]
    nvec, dvec = batched_er_sizes(512)
    torch.cuda.synchronize()
    log(f"batched: generated and uploaded 512 problems in {time.time() - t:.1f}s")
    res = {"workload": "512 ER products, n_i log-uniform in [2^10,2^17], d_i in {2..32}, values U[-1,1)"}
    for prec in ("f64", "f32c"):
        cache = {}

        def prepared(tune):
            key = (tune["tile_tuples"], tune["expand_chunk"])
            if key not in cache:
                cache.clear()
                cache[key] = _batch_plan(pb, torch, pairs, prec, tune)
            return cache[key]

        outs = None

        def run(tune):
            nonlocal outs
            sym, plan, ws = prepared(tune)
            if outs is None:
                outs = _outputs(torch, pairs, plan.flops, prec)
            pb.spgemm_batched(plan, pairs, ws, outs, sync=True)

        key = autotune.size_class(512, (dvec * dvec * nvec).tolist(), int(nvec.max()), prec)
        best = autotune.tune(run, key, log=log)
        tune = {"tile_tuples": best["tile_tuples"], "expand_chunk": best["expand_chunk"]}
        sym, plan, ws = prepared(tune)
        if outs is None:  # the tuning came from the cache, nothing ran yet
            outs = _outputs(torch, pairs, plan.flops, prec)
        nnz = pb.spgemm_batched(plan, pairs, ws, outs, sync=True)
        tot_flop = int(sum(plan.flops))
        tot_nnz = int(sum(nnz))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            p2 = pb.spgemm_batched_symbolic(pairs, prec, tune, sym_ws=sym)
            pb.spgemm_batched(p2, pairs, ws, outs, sync=False)
            p2.close()
        torch.cuda.synchronize()
        whole = (time.perf_counter() - t0) / steps
        graph_ms = _graph_ms(torch, lambda st: pb.spgemm_batched(plan, pairs, ws, outs, sync=False, stream=st),
                             steps, warmup)
        mb = sum(model_bytes(a.nrows, a.ncols, a.nnz, b.nnz, f, 0, prec)["total"]
                 for (a, b), f in zip(pairs, plan.flops)) + (12 if prec == "f64" else 8) * tot_nnz
        res[prec] = {"tune": tune, "autotune_cached": best.get("cached"), "autotune_timings_ms": best.get("timings_ms"),
                     "flop": tot_flop, "nnz_c": tot_nnz,
                     "whole_path_ms": round(whole * 1e3, 3), "whole_path_GFLOPS": round(2 * tot_flop / whole / 1e9, 2),
                     "numeric_graph_ms": round(graph_ms, 3),
                     "numeric_graph_GFLOPS": round(2 * tot_flop / (graph_ms * 1e-3) / 1e9, 2),
                     "model_GB": round(mb / 1e9, 2),
                     "numeric_graph_model_GBps": round(mb / (graph_ms * 1e-3) / 1e9, 1),
                     "numeric_graph_frac_of_8TBps": round(mb / (graph_ms * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4)}
        log(f"batched {prec}: {res[prec]['whole_path_GFLOPS']} GFLOPS whole path, "
            f"{res[prec]['numeric_graph_GFLOPS']} GFLOPS numeric graph")
        flops = list(plan.flops)
        cache.clear()
        del sym, plan, ws
        torch.cuda.empty_cache()
        # the same batch cut into flop size classes, each class its own
        # block-diagonal batch with its own tuned tile and expand chunk
        cb = autotune.ClassedBatch(pairs, prec, flops)
        chosen = cb.choose(outs, log=log)
        cb.run(outs, sync=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            cb.symbolic()
            cb.run(outs, sync=False)
        torch.cuda.synchronize()
        whole_c = (time.perf_counter() - t0) / steps
        graph_c = _graph_ms(torch, lambda st: cb.run(outs, sync=False, stream=st), steps, warmup)
        cb.close()
        res[prec]["size_classes"] = {
            "flop_bounds": list(autotune.SIZE_BOUNDS),
            "classes": [{"count": ch["count"], "flop": ch["flop"],
                         "tune": {"tile_tuples": ch["tile_tuples"], "expand_chunk": ch["expand_chunk"]},
                         "autotune_cached": ch.get("cached")} for ch in chosen],
            "whole_path_ms": round(whole_c * 1e3, 3), "whole_path_GFLOPS": round(2 * tot_flop / whole_c / 1e9, 2),
            "numeric_graph_ms": round(graph_c, 3),
            "numeric_graph_GFLOPS": round(2 * tot_flop / (graph_c * 1e-3) / 1e9, 2)}
        log(f"batched {prec} by size class: {res[prec]['size_classes']['whole_path_GFLOPS']} GFLOPS whole path, "
            f"{res[prec]['size_classes']['numeric_graph_GFLOPS']} GFLOPS numeric graph")
        del outs, cb
        outs = None
        torch.cuda.empty_cache()
    # the plain FP64 path, one product at a time, everything preallocated
    plans = []
    for a, b in pairs:
        nsym = pb.spgemm_symbolic(a, b, "f64")
        sym = torch.empty(max(nsym, 1), dtype=torch.uint8, device="cuda")
        plans.append((sym, pb.spgemm_symbolic(a, b, "f64", sym_ws=sym)))
    ws = torch.empty(max(p.workspace_bytes for _, p in plans), dtype=torch.uint8, device="cuda")
    outs = _outputs(torch, pairs, [p.flop for _, p in plans], "f64")
    for (a, b), (sym, p), o in zip(pairs, plans, outs):
        pb.spgemm_numeric(p, a, b, ws, *o, sync=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for (a, b), (sym, _), o in zip(pairs, plans, outs):
            p = pb.spgemm_symbolic(a, b, "f64", sym_ws=sym)
            pb.spgemm_numeric(p, a, b, ws, *o, sync=False)
            p.close()
    torch.cuda.synchronize()
    seq = (time.perf_counter() - t0) / steps

    def seq_numeric(st):
        for (a, b), (_, p), o in zip(pairs, plans, outs):
            pb.spgemm_numeric(p, a, b, ws, *o, sync=False, stream=st)

    seq_graph = _graph_ms(torch, seq_numeric, steps, warmup)
    for _, p in plans:
        p.close()
    del plans, ws, outs
    torch.cuda.empty_cache()
    flop = res["f64"]["flop"]
    res["sequential_f64"] = {"note": "plain path, one product at a time, plans/workspace/outputs preallocated",
                             "whole_path_ms": round(seq * 1e3, 2), "whole_path_GFLOPS": round(2 * flop / seq / 1e9, 2),
                             "numeric_graph_ms": round(seq_graph, 3),
                             "numeric_graph_GFLOPS": round(2 * flop / (seq_graph * 1e-3) / 1e9, 2)}
    for prec in ("f64", "f32c"):
        res[f"speedup_batched_{prec}_vs_sequential_f64"] = {
            "whole_path": round(seq / (res[prec]["whole_path_ms"] * 1e-3), 3),
            "numeric_graph": round(seq_graph / res[prec]["numeric_graph_ms"], 3)}
        sc = res[prec]["size_classes"]
        res[f"speedup_size_classes_{prec}_vs_sequential_f64"] = {
            "whole_path": round(seq / (sc["whole_path_ms"] * 1e-3), 3),
            "numeric_graph": round(seq_graph / sc["numeric_graph_ms"], 3)}
    res["speedup_batched_f32c_vs_batched_f64"] = {
        "whole_path": round(res["f64"]["whole_path_ms"] / res["f32c"]["whole_path_ms"], 3),
        "numeric_graph": round(res["f64"]["numeric_graph_ms"] / res["f32c"]["numeric_graph_ms"], 3)}
    log(f"batched: sequential FP64 {seq * 1e3:.1f} ms whole path, {seq_graph:.1f} ms numeric graph")
    return res


def bench_amg(pb, torch, steps, warmup):
    """AMG Galerkin chain on the 128^3 7-point Laplacian: T = A*P, Ac = R*T,
    each product's symbolic and numeric step, every buffer allocated
    beforehand.  T's nnz is read back (one sync) because it sizes the second
    product's operand."""
    from workloads import Csx, amg_problem

    A, P = amg_problem(128)
    Ad = pb.DeviceCsx.from_host(Csx(A.nrows, A.ncols, A.ptr, A.idx, A.val, "csc"))
    Pd = pb.DeviceCsx.from_host(P)
    Rd = Pd.transpose_view()
    res = {"workload": "AMG R*(A*P), 7-point Laplacian 128^3, smoothed aggregation 2x2x2, omega=2/3"}
    for prec in ("f64", "f32c"):
        vdt = torch.float64 if prec == "f64" else torch.float32
        s1 = torch.empty(pb.spgemm_symbolic(Ad, Pd, prec), dtype=torch.uint8, device="cuda")
        p1 = pb.spgemm_symbolic(Ad, Pd, prec, sym_ws=s1)
        T = (torch.empty(Ad.nrows + 1, dtype=torch.int64, device="cuda"),
             torch.empty(p1.flop, dtype=torch.int32, device="cuda"), torch.empty(p1.flop, dtype=vdt, device="cuda"))
        ws1 = torch.empty(p1.workspace_bytes, dtype=torch.uint8, device="cuda")
        nnz_t = pb.spgemm_numeric(p1, Ad, Pd, ws1, *T)
        Tval64 = torch.empty(nnz_t, dtype=torch.float64, device="cuda")
        Td = pb.DeviceCsx(Ad.nrows, Pd.ncols, T[0], T[1][:nnz_t], Tval64)
        Tval64.copy_(T[2][:nnz_t])
        s2 = torch.empty(pb.spgemm_symbolic(Rd, Td, prec), dtype=torch.uint8, device="cuda")
        p2 = pb.spgemm_symbolic(Rd, Td, prec, sym_ws=s2)
        Ac = (torch.empty(Rd.nrows + 1, dtype=torch.int64, device="cuda"),
              torch.empty(p2.flop, dtype=torch.int32, device="cuda"), torch.empty(p2.flop, dtype=vdt, device="cuda"))
        ws2 = torch.empty(p2.workspace_bytes, dtype=torch.uint8, device="cuda")
        flop = p1.flop + p2.flop
        p1.close()
        p2.close()

        def chain():
            q1 = pb.spgemm_symbolic(Ad, Pd, prec, sym_ws=s1)
            n1 = pb.spgemm_numeric(q1, Ad, Pd, ws1, *T)  # syncs: nnz(T) sizes the next operand
            q1.close()
            if prec == "f64":
                tv = T[2][:n1]
            else:  # operands are double: the float T is widened
                tv = Tval64[:n1]
                tv.copy_(T[2][:n1])
            Tn = pb.DeviceCsx(Ad.nrows, Pd.ncols, T[0], T[1][:n1], tv)
            q2 = pb.spgemm_symbolic(Rd, Tn, prec, sym_ws=s2)
            pb.spgemm_numeric(q2, Rd, Tn, ws2, *Ac, sync=False)
            q2.close()

        for _ in range(warmup):
            chain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            chain()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        nnz_ac = int(Ac[0][-1].item())
        res[prec] = {"chain_ms": round(dt * 1e3, 3), "GFLOPS": round(2 * flop / dt / 1e9, 2), "flop": flop,
                     "nnz_T": nnz_t, "nnz_Ac": nnz_ac}
        log(f"amg {prec}: {dt * 1e3:.3f} ms per chain")
        del T, Ac, ws1, ws2, s1, s2, Tval64
        torch.cuda.empty_cache()
    res["f32c_speedup_vs_f64"] = round(res["f64"]["chain_ms"] / res["f32c"]["chain_ms"], 3)
    return res


def run_rounds(pb, plan, A, B, ws, out, nrounds, count=False):
    """All rounds of a plan into one reused output buffer (as a consumer that
    streams C out would); with count, synchronise after each round and
    return nnz(C)."""
    rp, ci, cv = out
    total = 0
    for r in range(nrounds):
        nnz = pb.spgemm_numeric_round(plan, A, B, r, ws, rp, ci, cv, sync=count)
        if count:
            total += nnz
    return total


def prepare_rounds(pb, torch, A, B, prec, tune):
    """Symbolic step, round cut, workspace and one round's output buffers."""
    nsym = pb.spgemm_symbolic(A, B, prec, tune)
    sym = torch.empty(nsym, dtype=torch.uint8, device="cuda")
    plan = pb.spgemm_symbolic(A, B, prec, tune, sym_ws=sym)
    rb, fl = pb.spgemm_plan_rounds(plan)
    ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
    maxrows = max(rb[i + 1] - rb[i] for i in range(len(fl)))
    out = (torch.empty(maxrows + 1, dtype=torch.int64, device="cuda"),
           torch.empty(max(fl), dtype=torch.int32, device="cuda"),
           torch.empty(max(fl), dtype=torch.float64 if prec == "f64" else torch.float32, device="cuda"))
    return plan, sym, ws, out, len(fl)


def bench_rmat(pb, torch, steps, warmup, scale=20, edge_factor=16, round_tuples=1 << 32):
    """R-MAT C = A*A (symmetric A: its CSR arrays are its CSC arrays).  Its
    tuples and C exceed device memory, so the product runs as row-range
    rounds, each round's C going to one reused buffer; wide (hub) rows go
    through the column windows.  Sampled rows of this product are checked
    against the oracle by the GPU tests."""
    from workloads import rmat_symmetric

    t = time.time()
    a = rmat_symmetric(scale, edge_factor)
    ac = a.transpose_view()
    log(f"generated R-MAT scale {scale} ef {edge_factor}: nnz {a.nnz} in {time.time() - t:.1f}s")
    A = pb.DeviceCsx.from_host(ac)
    B = pb.DeviceCsx.from_host(a)
    res = {"workload": f"R-MAT scale {scale}, edge factor {edge_factor}, (a,b,c,d)=(.57,.19,.19,.05), symmetrized, "
                       f"values U[0,1), C=A*A", "nnz_a": a.nnz, "round_tuples": round_tuples}
    base_sec = None
    for prec in ("f64", "f32c"):
        tune = {"round_tuples": round_tuples}
        plan, sym, ws, out, nr = prepare_rounds(pb, torch, A, B, prec, tune)
        flop = plan.flop
        log(f"rmat {prec}: flop {flop}, {nr} rounds, workspace {plan.workspace_bytes / 1e9:.1f} GB")
        nnz_c = run_rounds(pb, plan, A, B, ws, out, nr, count=True)
        plan.close()

        def step():
            p = pb.spgemm_symbolic(A, B, prec, tune, sym_ws=sym)
            run_rounds(pb, p, A, B, ws, out, nr)
            p.close()

        sec, prof = time_steps(torch, pb, step, steps, warmup)
        res[prec] = {"GFLOPS": round(2.0 * flop / sec / 1e9, 3), "ms_per_product": round(sec * 1e3, 2),
                     "phases_ms_per_product": {k: round(ms / max(steps, 1), 3) for k, (ms, n) in prof.items()},
                     "flop": flop, "nnz_c": nnz_c, "rounds": nr}
        log(f"rmat {prec}: {sec * 1e3:.1f} ms per product, {2.0 * flop / sec / 1e9:.1f} GFLOPS, nnz(C) {nnz_c}")
        if prec == "f64":
            base_sec = sec
        else:
            res["f32c_speedup_vs_f64"] = round(base_sec / sec, 3)
        del ws, out, sym
        torch.cuda.empty_cache()
    res["f32c_error_vs_f64_by_round"] = rmat_f32c_error(pb, torch, A, B, round_tuples)
    return res


def rmat_f32c_error(pb, torch, A, B, round_tuples):
    """FP32c against FP64 on two rounds of the R-MAT product (the lightest
    and a middle one).  Both plans use run alignment 1, so their rounds cover
    the same rows; values are U[0,1), so N = C."""
    tune = {"round_tuples": round_tuples, "run_align": 1}
    kept, out_err = {}, []
    for prec in ("f64", "f32c"):
        plan, sym, ws, out, nr = prepare_rounds(pb, torch, A, B, prec, tune)
        rb, fl = pb.spgemm_plan_rounds(plan)
        for r in sorted({int(np.argmin(fl)), nr // 2}):
            n = pb.spgemm_numeric_round(plan, A, B, r, ws, *out)
            rows = rb[r + 1] - rb[r]
            if prec == "f64":
                kept[r] = (rb[r], rows, out[0][: rows + 1].clone(), out[1][:n].clone(), out[2][:n].clone())
                continue
            r0, rows64, rp, ci, cv = kept.pop(r)
            assert r0 == rb[r] and rows64 == rows, "rounds differ between precisions"
            assert torch.equal(rp, out[0][: rows + 1]) and torch.equal(ci, out[1][:n]), "FP32c structure differs"
            nz = cv != 0
            rel = (out[2][:n].double() - cv).abs()[nz] / cv.abs()[nz]
            out_err.append({"round": r, "rows": rows, "nnz": n,
                            "f32c_max_err_over_N": float(rel.max().item()) if rel.numel() else 0.0})
            del rp, ci, cv, rel
        plan.close()
        del ws, out, sym
        torch.cuda.empty_cache()
    return out_err


SWEEP_ER = [(s, d) for s in (16, 18, 20, 22) for d in (4, 8, 16, 32)]
SWEEP_RMAT = [(s, ef) for s in (16, 18, 20) for ef in (4, 8, 16)]


def sweep_inputs(family, scale, ef):
    """A (CSC) and B (CSR) of one sweep point: ER A*B with the seeds of the
    n=2^20 workload, or R-MAT A*A."""
    from workloads import er_problem, rmat_symmetric

    if family == "er":
        return er_problem(1 << scale, ef, 2, 3)
    r = rmat_symmetric(scale, ef)
    return r.transpose_view(), r


def sweep_case(pb, torch, family, scale, ef, beta, tune_path, target_s=0.4):
    """One point of the scale x edge-factor sweep, FP64: whole-path time,
    the byte model beside it and, for products whose C fits whole, the
    autotuner's tile and chunk choice.  Products above 2^32 tuples run as
    row-range rounds into one reused buffer."""
    from paper_2002_11302_amd import autotune

    prec = "f64"
    t = time.time()
    a, b = sweep_inputs(family, scale, ef)
    t_gen = time.time() - t
    A, B = pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)
    flop = int(np.dot(np.diff(a.ptr), np.diff(b.ptr)))
    rounds = flop > (1 << 32)
    if rounds:
        tune = {"round_tuples": 1 << 32}
        plan, sym, ws, out, nr = prepare_rounds(pb, torch, A, B, prec, tune)
        info = plan.info()
        nnz_c = run_rounds(pb, plan, A, B, ws, out, nr, count=True)
        plan.close()

        def step():
            p = pb.spgemm_symbolic(A, B, prec, tune, sym_ws=sym)
            run_rounds(pb, p, A, B, ws, out, nr)
            p.close()
    else:
        nr = 1
        nsym = pb.spgemm_symbolic(A, B, prec, None)
        sym = torch.empty(nsym, dtype=torch.uint8, device="cuda")
        plan = pb.spgemm_symbolic(A, B, prec, None, sym_ws=sym)
        info = plan.info()
        ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
        out = (torch.empty(a.nrows + 1, dtype=torch.int64, device="cuda"),
               torch.empty(max(flop, 1), dtype=torch.int32, device="cuda"),
               torch.empty(max(flop, 1), dtype=torch.float64, device="cuda"))
        nnz_c = pb.spgemm_numeric(plan, A, B, ws, *out, sync=True)
        plan.close()

        def step():
            p = pb.spgemm_symbolic(A, B, prec, None, sym_ws=sym)
            pb.spgemm_numeric(p, A, B, ws, *out, sync=False)
            p.close()

    assert info["flop"] == flop
    t0 = time.perf_counter()
    step()
    torch.cuda.synchronize()
    est = time.perf_counter() - t0
    steps = int(min(50, max(2, target_s / max(est, 1e-6))))
    sec, prof = time_steps(torch, pb, step, steps, 1)
    mb = model_bytes(a.nrows, a.ncols, a.nnz, b.nnz, flop, nnz_c, prec)
    res = {"family": family, "scale": scale, "edge_factor": ef, "nnz_a": a.nnz, "nnz_b": b.nnz, "flop": flop,
           "nnz_c": int(nnz_c), "cf": round(flop / max(nnz_c, 1), 3), "max_row_flop": info["max_row_flop"],
           "tile_tuples": info["tile_tuples"], "expand_chunk": info["expand_chunk"], "nbins": info["nbins"],
           "rounds": nr, "steps": steps, "ms": round(sec * 1e3, 3),
           "GFLOPS": round(2.0 * flop / sec / 1e9, 2),
           "phases_ms": {k: round(ms / steps, 3) for k, (ms, n) in prof.items()},
           "model_GB": round(mb["total"] / 1e9, 4), "model_GBps": round(mb["total"] / sec / 1e9, 1),
           "frac_beta": round(mb["total"] / sec / 1e9 / beta, 4),
           "model_GFLOPS_at_beta": round(2.0 * flop / (mb["total"] / (beta * 1e9)) / 1e9, 1),
           "paper_b16_GFLOPS_at_beta": round(2.0 * flop / (mb["paper_b16"] / (beta * 1e9)) / 1e9, 1),
           "generate_s": round(t_gen, 1)}
    if not rounds:
        need = 0
        for cand in autotune.CANDIDATES:
            try:
                p = pb.spgemm_symbolic(A, B, prec, cand, sym_ws=sym)
            except pb.PbError:
                continue  # the tuner skips candidates the library rejects
            need = max(need, p.workspace_bytes)
            p.close()
        del ws
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")

        def run(cand):
            p = pb.spgemm_symbolic(A, B, prec, cand, sym_ws=sym)
            pb.spgemm_numeric(p, A, B, ws, *out, sync=True)
            p.close()

        choice = autotune.tune(run, f"sweep|{family}|s{scale}|ef{ef}|{prec}", reps=2, path=tune_path)
        res["autotune"] = {"tile_tuples": choice["tile_tuples"], "expand_chunk": choice["expand_chunk"],
                           "timings_ms": choice["timings_ms"]}
    del ws, out, sym, A, B
    torch.cuda.empty_cache()
    return res


def bench_sweep(pb, torch, beta, tune_path):
    out = []
    for family, grid in (("er", SWEEP_ER), ("rmat", SWEEP_RMAT)):
        for scale, ef in grid:
            log(f"sweep {family} scale {scale} ef {ef}")
            r = sweep_case(pb, torch, family, scale, ef, beta, tune_path)
            log(f"sweep {family} scale {scale} ef {ef}: {r['ms']} ms, {r['GFLOPS']} GFLOPS, "
                f"{r['model_GBps']} GB/s model ({100 * r['frac_beta']:.1f}% of copy), cf {r['cf']}, "
                f"{r['rounds']} round(s)"
                + (f", tuned T{r['autotune']['tile_tuples']} C{r['autotune']['expand_chunk']}"
                   if "autotune" in r else ""))
            out.append(r)
    return out


def summarize_profiles(src: str, out_dir: str, command: str, pmc_command: str) -> None:
    """Turn rocprofv3 CSV output (kernel trace stats and two counter runs,
    FETCH_SIZE then WRITE_SIZE) into the text summaries under profiles/ and
    the per-launch HBM traffic table bench.py reports.  The counters are
    scaled by what they read for the 16-byte copy kernel of known size."""
    import csv
    import glob

    def rows(pattern):
        files = glob.glob(os.path.join(src, pattern), recursive=True)
        if not files:
            raise FileNotFoundError(pattern)
        with open(files[0]) as f:
            return list(csv.DictReader(f))

    def short(name):
        for key in ("k_expand", "k_sort_compress_fused", "k_sort_compress", "k_row_nnz", "k_rowflop",
                    "k_bucket_hist", "k_bucket_scatter", "k_bucket_count", "k_bucket_dest", "k_bucket_offsets",
                    "k_entry_dest", "k_bin_max", "k_scan_tiles", "k_scan_apply", "k_chunk_start", "k_copy16",
                    "k_fill_u32", "k_pack"):
            if key in name:
                prec = "f32c" if "float" in name else ("f64" if "double" in name else "")
                return f"{key}<{prec}>" if prec else key
        return name[:40]

    stats = rows("kt/**/*kernel_stats.csv")
    lines = [f"# rocprofv3 kernel-trace summary: ER n=2^20 d=16 A*B (bench.py workload)",
             f"# command: {command}",
             f"# {'kernel':58s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for r in stats:
        lines.append(f"  {r['Name'][:58]:58s} {r['Calls']:>6s} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f}")
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, "kernels_er2e20_d16.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")

    def per_kernel(kind):
        acc = {}
        for r in rows(f"{kind}/**/*counter_collection.csv"):
            if r.get("Counter_Name") != kind.upper() + "_SIZE":
                continue
            k = short(r["Kernel_Name"])
            acc.setdefault(k, []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    fetch, write = per_kernel("fetch"), per_kernel("write")
    copy_bytes = 4 << 30
    f_scale = copy_bytes / (fetch["k_copy16"] * 1024.0)
    w_scale = copy_bytes / (write["k_copy16"] * 1024.0)
    sha = kernel_source_sha()
    traffic = {"_calibration": {"copy_bytes": copy_bytes, "fetch_scale": f_scale, "write_scale": w_scale,
                                "kernel_source_sha256": sha}}
    lines = ["# HBM traffic per launch from rocprofv3 counters (FETCH_SIZE and WRITE_SIZE, KiB per dispatch),",
             f"# scaled by the copy kernel: fetch x{f_scale:.3f}, write x{w_scale:.3f} (4 GiB copy reads and writes 4 GiB)",
             "# commands: " + pmc_command.replace("{COUNTER}", "FETCH_SIZE").replace("{KIND}", "fetch"),
             "#      and: " + pmc_command.replace("{COUNTER}", "WRITE_SIZE").replace("{KIND}", "write"),
             f"# {'kernel':28s} {'fetch_KiB':>14s} {'write_KiB':>14s} {'fetch_GB':>10s} {'write_GB':>10s}"]
    for k in sorted(set(fetch) | set(write)):
        fb = fetch.get(k, 0.0) * 1024 * f_scale
        wb = write.get(k, 0.0) * 1024 * w_scale
        lines.append(f"  {k:28s} {fetch.get(k, 0.0):14.1f} {write.get(k, 0.0):14.1f} {fb / 1e9:10.3f} {wb / 1e9:10.3f}")
        if k.startswith(("k_expand", "k_sort_compress", "k_row_nnz")):
            traffic[k] = {"bytes_per_launch": int(fb + wb), "fetch_bytes": int(fb), "write_bytes": int(wb),
                          "kernel_source_sha256": sha}
    with open(os.path.join(out_dir, "hbm_traffic_er2e20_d16.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    with open(os.path.join(out_dir, "traffic.json"), "w") as f:
        json.dump(traffic, f, indent=1, sort_keys=True)
        f.write("\n")


def summarize_rmat_counters(src: str, out_path: str, pmc_command: str) -> None:
    """Write the R-MAT product's HBM traffic per kernel and product from two
    rocprofv3 counter runs (FETCH_SIZE then WRITE_SIZE in src/fetch and
    src/write) of `bench.py --quick --rmat`, scaled by what the counters read
    for the copy kernel.  That run does, per precision, four products (one
    to count nnz(C), one warm-up, two timed): kernels templated on the value
    type ran in 4 products, the others in 8 (the ER n=2^20 steps that run
    first add well under 1 % of these bytes)."""
    import csv
    import glob

    def per_kernel(kind):
        files = glob.glob(os.path.join(src, kind, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise FileNotFoundError(f"no counter_collection.csv under {src}/{kind}")
        acc, n = {}, {}
        with open(files[0]) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != kind.upper() + "_SIZE":
                    continue
                name = r["Kernel_Name"]
                key = name.split("(")[0].replace("void ", "").strip()
                if "double" in name:
                    key += " <f64>"
                elif "float" in name:
                    key += " <f32c>"
                acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
                n[key] = n.get(key, 0) + 1
        return acc, n

    (fetch, nf), (write, _) = per_kernel("fetch"), per_kernel("write")
    copy_bytes = 4 << 30
    copy = [k for k in fetch if "k_copy16" in k][0]
    f_scale = copy_bytes / (fetch[copy] / nf[copy] * 1024.0)
    w_scale = copy_bytes / (write[copy] / nf[copy] * 1024.0)
    lines = ["# HBM traffic per R-MAT product (scale 20, ef 16, C = A*A in 17 rounds) from rocprofv3 counters",
             f"# (FETCH_SIZE and WRITE_SIZE summed over a kernel's dispatches, divided by the products that ran it),",
             f"# scaled by the copy kernel: fetch x{f_scale:.3f}, write x{w_scale:.3f}",
             "# commands: " + pmc_command.replace("{COUNTER}", "FETCH_SIZE").replace("{KIND}", "fetch"),
             "#      and: " + pmc_command.replace("{COUNTER}", "WRITE_SIZE").replace("{KIND}", "write"),
             f"# {'kernel':56s} {'dispatches':>10s} {'fetch_GB':>10s} {'write_GB':>10s}  (per product)"]
    items = []
    for k in set(fetch) | set(write):
        if "k_copy16" in k or not k.startswith("pb::"):
            continue  # the product's own kernels only (not the host-side checks' torch kernels)
        prods = 4 if k.endswith(("<f64>", "<f32c>")) else 8
        fb = fetch.get(k, 0.0) * 1024 * f_scale / prods
        wb = write.get(k, 0.0) * 1024 * w_scale / prods
        items.append((fb + wb, k, nf.get(k, 0), fb, wb))
    for _, k, nd, fb, wb in sorted(items, reverse=True):
        if fb + wb < 1e8:
            continue
        lines.append(f"  {k[:56]:56s} {nd:10d} {fb / 1e9:10.2f} {wb / 1e9:10.2f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize_trace(src: str, out_path: str, title: str, command: str, per=lambda name: 1) -> None:
    """Write a rocprofv3 kernel-trace stats summary (the kernels of src's
    kernel_stats.csv, longest first, with the time per product when the
    traced run did per(kernel name) products with that kernel)."""
    import csv
    import glob

    files = glob.glob(os.path.join(src, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no kernel_stats.csv under {src}")
    with open(files[0]) as f:
        stats = sorted(csv.DictReader(f), key=lambda r: -float(r["TotalDurationNs"]))
    lines = [f"# rocprofv3 kernel-trace summary: {title}", f"# command: {command}",
             f"# {'kernel':70s} {'calls':>6s} {'avg_us':>10s} {'total_ms':>10s} {'ms_per_product':>14s} {'pct':>6s}"]
    for r in stats:
        tot = float(r["TotalDurationNs"]) / 1e6
        lines.append(f"  {r['Name'][:70]:70s} {r['Calls']:>6s} {float(r['AverageNs']) / 1e3:10.2f} {tot:10.3f} "
                     f"{tot / per(r['Name']):14.3f} {float(r['Percentage']):6.2f}")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["f64", "f32c"], default="f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true",
                    help="only the headline product (skip the FP32c, AMG, batched and R-MAT legs)")
    ap.add_argument("--extras", action="store_true", help="with --quick: the FP32c leg")
    ap.add_argument("--batched", action="store_true", help="with --quick: the 512-product batched leg")
    ap.add_argument("--amg", action="store_true", help="with --quick: the AMG Galerkin chain leg")
    ap.add_argument("--rmat", action="store_true",
                    help="with --quick: the R-MAT scale 20 C=A*A leg (row-range rounds, wide rows), FP64 and FP32c")
    ap.add_argument("--sweep", action="store_true",
                    help="also run the scale x edge-factor sweep (ER A*B and R-MAT A*A, FP64) with the byte model, "
                         "sampled-row parity and the autotuner's choice per point")
    ap.add_argument("--summarize-profiles", metavar="DIR", help="write profiles/ summaries from rocprofv3 output in DIR")
    ap.add_argument("--profile-command", default="", help="the kernel-trace command, recorded in the summaries")
    ap.add_argument("--summarize-rmat-trace", metavar="DIR",
                    help="write profiles/kernels_rmat_s20_ef16.txt from a rocprofv3 kernel trace of "
                         "`bench.py --rmat --steps 2 --warmup 1 --no-cpu-baseline` in DIR")
    ap.add_argument("--summarize-rmat-counters", metavar="DIR",
                    help="write profiles/hbm_traffic_rmat_s20_ef16.txt from FETCH_SIZE and WRITE_SIZE runs of "
                         "`bench.py --quick --rmat --no-cpu-baseline` in DIR/fetch and DIR/write")
    ap.add_argument("--pmc-command", default="",
                    help="the counter command, with {COUNTER} and {KIND} for FETCH_SIZE/fetch and WRITE_SIZE/write")
    args = ap.parse_args()
    if args.summarize_rmat_trace:
        # that run does, per precision, one product to count nnz(C), one
        # warm-up and two timed products: kernels templated on the value
        # type ran in 4 products, the others in 8 (the ER n=2^20 steps that
        # run first are a few ms against seconds)
        summarize_trace(args.summarize_rmat_trace, os.path.join(ROOT, "profiles", "kernels_rmat_s20_ef16.txt"),
                        "R-MAT scale 20 ef 16 C = A*A, FP64 and FP32c, 4 products each (plus the ER n=2^20 d=16 "
                        "steps bench.py runs first)", args.profile_command,
                        per=lambda name: 4 if ("double" in name or "float" in name) else 8)
        return
    if args.summarize_rmat_counters:
        summarize_rmat_counters(args.summarize_rmat_counters,
                                os.path.join(ROOT, "profiles", "hbm_traffic_rmat_s20_ef16.txt"), args.pmc_command)
        return
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, os.path.join(ROOT, "profiles"), args.profile_command,
                           args.pmc_command)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the product has no multi-GPU path; "
              "value is one GPU's throughput.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2002_11302_amd as pb

    pb.load()
    assert torch.cuda.is_available(), "needs a GPU"
    a, b, A, B = build_inputs(pb, torch)
    step, flop, rowptr_c = make_step(pb, torch, A, B, args.precision)
    rowptr = rowptr_c[0]
    log(f"flop={flop}; timing {args.steps} steps after {args.warmup} warm-up")
    sec, prof = time_steps(torch, pb, step, args.steps, args.warmup)
    nnz_c = int(rowptr[-1].item())
    mb = model_bytes(a.nrows, a.ncols, a.nnz, b.nnz, flop, nnz_c, args.precision)
    phase_ms = {k: (ms / max(n, 1)) for k, (ms, n) in prof.items()}
    log("phase avg ms: " + ", ".join(f"{k}={v:.4f}" for k, v in phase_ms.items()))
    dom = max(("expand", "sort_compress"), key=lambda k: phase_ms[k])
    achieved = mb[dom] / (phase_ms[dom] * 1e-3) / 1e9
    kernel_key = {"expand": f"k_expand<{args.precision}>", "sort_compress": f"k_sort_compress<{args.precision}>"}[dom]
    value = 2.0 * flop / sec / 1e9
    out = {
        "metric": "effective GFLOPS (2*flop/s), PB-SpGEMM whole path (symbolic + numeric)",
        "value": round(value, 3),
        "unit": "GFLOPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": "Erdos-Renyi A*B, n=2^20, 16 nonzeros per column, values U[0,1), C=A*B",
                   "m": a.nrows, "k": a.ncols, "n": b.ncols, "nnz_a": a.nnz, "nnz_b": b.nnz,
                   "flop": flop, "nnz_c": nnz_c, "precision": args.precision},
        "roofline": {"bound": "hbm", "kernel": kernel_key, "achieved": round(achieved, 1), "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBPS, 4), "traffic": traffic_for(kernel_key),
                     "algorithmic_bytes_per_launch": mb[dom], "avg_launch_ms": round(phase_ms[dom], 5)},
        "phases_ms": {k: round(v, 5) for k, v in phase_ms.items()},
        "model_bytes": mb,
        "whole_path_model_GBps": round(mb["total"] / sec / 1e9, 1),
        "paper_MFLOPS": round(flop / sec / 1e6, 1),  # the paper's unit: multiplications per second
        "phase_model_GBps": {k: round(mb[k] / (phase_ms[k] * 1e-3) / 1e9, 1) for k in ("expand", "sort_compress")},
    }
    amp = {}
    for k in ("expand", "sort_compress"):
        t = traffic_for(f"k_{k}<{args.precision}>")
        if t:
            amp[k] = round(t / mb[k], 3)
    out["traffic_over_model"] = amp or None
    beta = copy_bandwidth(pb, torch)
    out["copy_GBps"] = round(beta, 1)
    out["roofline"]["frac_of_copy"] = round(achieved / beta, 4)
    gpu_results = {args.precision: make_step_outputs(rowptr_c)}
    legs = {"f32c": args.extras, "amg": args.amg, "batched": args.batched, "rmat": args.rmat}
    if not args.quick:
        legs = {k: True for k in legs}
    ex = out.setdefault("extras", {})
    if legs["f32c"]:
        other = "f32c" if args.precision == "f64" else "f64"
        log(f"leg: {other} on the same product")
        step2, _, outs2 = make_step(pb, torch, A, B, other)
        sec2, prof2 = time_steps(torch, pb, step2, args.steps, args.warmup)
        gpu_results[other] = make_step_outputs(outs2)
        ex[other] = {"GFLOPS": round(2.0 * flop / sec2 / 1e9, 3), "ms_per_step": round(sec2 * 1e3, 4),
                     "phases_ms": {k: round(ms / max(n, 1), 5) for k, (ms, n) in prof2.items()},
                     f"speedup_vs_{args.precision}": round(sec / sec2, 3)}
        if other == "f32c":
            ex["f32c"]["error_vs_f64_over_N"] = fp32c_error(pb, torch, A, B, signed=False)
    if legs["amg"]:
        log("leg: AMG chain")
        ex["amg"] = bench_amg(pb, torch, max(3, args.steps // 4), 1)
        ex["amg"]["f32c_error_vs_f64_over_N"] = amg_f32c_error(pb, torch)
    if legs["batched"]:
        log("leg: batched")
        ex["batched"] = bench_batched(pb, torch, max(2, args.steps // 10), 1)
        ex["batched"]["f32c_error_vs_f64_over_N"] = batched_f32c_error(pb, torch)
    if legs["rmat"]:
        log("leg: R-MAT")
        ex["rmat"] = bench_rmat(pb, torch, 2, 1)
    if args.sweep:
        import tempfile

        beta = out["copy_GBps"]
        ex["sweep_copy_GBps"] = beta
        ex["sweep"] = bench_sweep(pb, torch, beta, os.path.join(tempfile.mkdtemp(), "autotune.json"))
    if not ex:
        del out["extras"]
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the host")
        out["cpu_baseline"], out["oracle_check_of_this_run"] = cpu_baseline(a, b, torch, gpu_results)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
