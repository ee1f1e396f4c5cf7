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


# ---------------------------------------------------------------- size classes
# A batch of uneven products is cut by each product's multiplication count
# into size classes; each class runs as its own block-diagonal batch (one
# launch per kernel for all its products) with the tile and expand chunk the
# tuner picked for that class, and all classes go on one stream, so a HIP
# graph captures the whole batch.
SIZE_BOUNDS = (1 << 20, 1 << 24)  # flop bounds between the classes


def size_classes(flops, bounds=SIZE_BOUNDS) -> list:
    """Indices of the products in each flop class, smallest class first;
    empty classes are left out."""
    groups = [[] for _ in range(len(bounds) + 1)]
    for i, f in enumerate(flops):
        groups[sum(int(f) >= b for b in bounds)].append(i)
    return [g for g in groups if g]


class ClassedBatch:
    """C_i = A_i * B_i for a list of (A_csc, B_csr) device pairs, cut into
    size classes by ``flops`` (each product's multiplication count, e.g. a
    batched plan's ``flops``).  ``tunes`` gives each class's tuning; without
    it :meth:`choose` times the candidates per class (cached like
    :func:`tune`).  Every class holds its own symbolic workspace, plan and
    numeric workspace."""

    def __init__(self, pairs, precision: str, flops, bounds=SIZE_BOUNDS, tunes=None):
        self.pairs = list(pairs)
        self.precision = precision
        self.flops = [int(f) for f in flops]
        self.groups = size_classes(self.flops, bounds)
        self.tunes = list(tunes) if tunes is not None else [None] * len(self.groups)
        if len(self.tunes) != len(self.groups):
            raise ValueError(f"{len(self.groups)} size classes but {len(self.tunes)} tunings")
        self._parts = [None] * len(self.groups)  # (tune, sym_ws, plan, workspace)
        for c, t in enumerate(self.tunes):
            if t is not None:
                self._prepare(c, t)

    def _sub(self, c, seq):
        return [seq[i] for i in self.groups[c]]

    def _prepare(self, c, tune_):
        from . import spgemm_batched_symbolic

        import torch

        part = self._parts[c]
        if part is not None and part[0] == tune_:
            return part
        if part is not None:
            part[2].close()
        sub = self._sub(c, self.pairs)
        dev = sub[0][0].ptr.device
        nsym = spgemm_batched_symbolic(sub, self.precision, tune_)
        sym = torch.empty(max(nsym, 1), dtype=torch.uint8, device=dev)
        plan = spgemm_batched_symbolic(sub, self.precision, tune_, sym_ws=sym)
        ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device=dev)
        self._parts[c] = (dict(tune_), sym, plan, ws)
        return self._parts[c]

    def choose(self, outs, reps: int = 3, path: str | None = None, log=None) -> list:
        """Pick every class's tile and expand chunk by timing the class
        into its outputs (``outs[i] = (rowptr, colidx, val)``)."""
        from . import spgemm_batched

        chosen = []
        for c, g in enumerate(self.groups):
            sub, subouts = self._sub(c, self.pairs), self._sub(c, outs)

            def run(t):
                _, _, plan, ws = self._prepare(c, {"tile_tuples": t["tile_tuples"],
                                                   "expand_chunk": t["expand_chunk"]})
                spgemm_batched(plan, sub, ws, subouts, sync=True)

            max_n = max(max(a.nrows, b.ncols) for a, b in sub)
            key = "class|" + size_class(len(g), [self.flops[i] for i in g], max_n, self.precision)
            best = tune(run, key, reps=reps, path=path, log=log)
            self.tunes[c] = {"tile_tuples": best["tile_tuples"], "expand_chunk": best["expand_chunk"]}
            self._prepare(c, self.tunes[c])
            chosen.append(dict(best, count=len(g), flop=sum(self.flops[i] for i in g)))
        return chosen

    def symbolic(self, stream=None) -> None:
        """Run every class's symbolic step again into its workspace (the
        plans are replaced; tunings and workspaces are kept)."""
        from . import spgemm_batched_symbolic

        for c, part in enumerate(self._parts):
            if part is None:
                raise RuntimeError("size class without a tuning: call choose() or pass tunes")
            t, sym, plan, ws = part
            plan.close()
            plan = spgemm_batched_symbolic(self._sub(c, self.pairs), self.precision, t, sym_ws=sym, stream=stream)
            self._parts[c] = (t, sym, plan, ws)

    def run(self, outs, sync: bool = True, stream=None):
        """Numeric step of every class into ``outs`` (in the batch's order).
        With ``sync`` returns every product's nnz(C); otherwise only
        enqueues (capturable in one HIP graph)."""
        from . import spgemm_batched

        nnz = [0] * len(self.pairs)
        for c, part in enumerate(self._parts):
            if part is None:
                raise RuntimeError("size class without a tuning: call choose() or pass tunes")
            _, _, plan, ws = part
            got = spgemm_batched(plan, self._sub(c, self.pairs), ws, self._sub(c, outs), sync=sync, stream=stream)
            if sync:
                for i, v in zip(self.groups[c], got):
                    nnz[i] = v
        return nnz if sync else None

    def close(self) -> None:
        for part in self._parts:
            if part is not None:
                part[2].close()
        self._parts = [None] * len(self.groups)
