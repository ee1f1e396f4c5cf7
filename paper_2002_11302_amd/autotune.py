"""Autotuner for the tile (bin width, hence bin count) and the expand chunk.

The sort tile T bounds the tuples per bin (so it sets the bin width and,
through the flop count, the number of bins) and selects the LDS sort kernel
variant; the expand chunk sets the tuples per expand wave.  For a workload
(one product or a batch) the tuner times every candidate through the same
entry points a user calls, keeps the fastest, and caches the choice in a
JSON file keyed by device, precision and a size class of the workload, so
later runs of workloads of the same class reuse it without timing.
"""
from __future__ import annotations

import json
import math
import os
import time

from . import _binding as _b

CANDIDATES = [
    {"tile_tuples": t, "expand_chunk": c} for t in (2048, 4096) for c in (512, 1024, 2048)
]


def cache_path() -> str:
    p = os.environ.get("PB_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "pbspgemm", "autotune.json")


def size_class(count: int, flops, max_n: int, precision: str) -> str:
    """Coarse signature: problem count, total flop and largest dimension on
    log2 scales."""
    tot = max(int(sum(flops)), 1)
    return f"{precision}|count{count}|flop2^{int(math.log2(tot))}|n2^{int(math.log2(max(max_n, 1)))}"


def _device_name() -> str:
    try:
        import torch

        return torch.cuda.get_device_properties(0).gcnArchName
    except Exception:
        return "unknown"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, data):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(run, key: str, candidates=None, reps: int = 3, path: str | None = None, log=None) -> dict:
    """Pick the fastest candidate for ``run(tune) -> None`` (which must do the
    work and synchronise).  Candidates the library rejects (for instance a
    tile smaller than the largest row) are skipped.  Returns the chosen tune
    dict, with the per-candidate timings under "timings_ms"."""
    path = path or cache_path()
    full_key = f"{_device_name()}|{key}"
    cache = _load(path)
    if full_key in cache:
        return dict(cache[full_key], cached=True)
    best, best_t, timings = None, float("inf"), {}
    for cand in candidates or CANDIDATES:
        name = f"T{cand['tile_tuples']}_C{cand['expand_chunk']}"
        try:
            run(cand)  # warm-up
            t0 = time.perf_counter()
            for _ in range(reps):
                run(cand)
            dt = (time.perf_counter() - t0) / reps
        except _b.PbError as e:
            if e.name in ("PB_ERR_UNSUPPORTED", "PB_ERR_ARG"):
                timings[name] = None
                continue
            raise
        timings[name] = round(dt * 1e3, 4)
        if log:
            log(f"autotune {name}: {dt * 1e3:.3f} ms")
        if dt < best_t:
            best, best_t = cand, dt
    if best is None:
        raise RuntimeError("no tuning candidate ran")
    entry = dict(best, timings_ms=timings)
    cache[full_key] = entry
    _store(path, cache)
    return dict(entry, cached=False)
