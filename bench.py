#!/usr/bin/env python3
"""Benchmark of the PB-SpGEMM hot path on one MI355X.

One step is the whole path for one product C = A*B: the symbolic step
(Algorithm 3's flop scan, per-row flop, bin cut; one host sync to size the
workspace) and the numeric step (expand into bins, per-bin LDS sort and
merge, CSR emission).  Inputs are resident in HBM before timing starts.

Workload (default): Erdos-Renyi A and B, n = 2^20, exactly 16 nonzeros per
column, values U[0,1) in double, C = A*B, FP64 path.

Prints ONE JSON line on stdout; progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--precision f64|f32c] [--no-cpu-baseline] [--extras]
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
    this build's widths: int64 pointers, int32 indices, double inputs, packed
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


def cpu_baseline(a, b):
    import oracle

    threads = len(os.sched_getaffinity(0))
    oracle.build(force=False)
    t = time.perf_counter()
    r = oracle.spgemm_cols(a, b, None, nthreads=threads)
    dt = time.perf_counter() - t
    flop = oracle.flop(a.ptr, b.ptr)
    del r
    return {"value": round(2.0 * flop / dt / 1e9, 4), "unit": "GFLOPS", "cores": threads, "kind": "oracle",
            "sample": f"full product: all {b.ncols} output columns of the ER n=2^20 d=16 A*B workload, FP64; "
                      f"{dt:.2f} s wall on {threads} host threads"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", choices=["f64", "f32c"], default="f64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", action="store_true", help="also time FP32c and the copy bandwidth")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (see DESIGN.md on sharding).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2002_11302_amd as pb

    pb.load()
    assert torch.cuda.is_available(), "needs a GPU"
    a, b, A, B = build_inputs(pb, torch)
    step, flop, (rowptr, _, _) = make_step(pb, torch, A, B, args.precision)
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
    }
    if args.extras:
        log("extras: FP32c step and copy bandwidth")
        other = "f32c" if args.precision == "f64" else "f64"
        step2, _, (rp2, _, _) = make_step(pb, torch, A, B, other)
        sec2, prof2 = time_steps(torch, pb, step2, args.steps, args.warmup)
        out["extras"] = {
            f"{other}_GFLOPS": round(2.0 * flop / sec2 / 1e9, 3),
            f"{other}_ms_per_step": round(sec2 * 1e3, 4),
            f"{other}_phases_ms": {k: round(ms / max(n, 1), 5) for k, (ms, n) in prof2.items()},
            "copy_GBps": round(copy_bandwidth(pb, torch), 1),
        }
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the host")
        out["cpu_baseline"] = cpu_baseline(a, b)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
