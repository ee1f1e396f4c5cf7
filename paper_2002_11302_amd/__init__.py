"""PB-SpGEMM on MI355X: Python binding of libpbspgemm.so.

C = A*B with A in CSC and B in CSR, emitted as CSR, by the outer-product
expand / bin / sort / compress method of Gu, Moreira, Edelsohn and Azad
(arXiv 2002.11302, Algorithms 2 and 3).  All arithmetic runs in the HIP
library; this module only moves pointers, sizes and torch-allocated device
memory across the C ABI, under the same names as the ABI's entry points.
"""
from __future__ import annotations

import ctypes
import dataclasses

from . import _binding as _b
from ._binding import NOALLOC_SCRATCH_BYTES, PHASES, PbError  # noqa: F401

__all__ = [
    "DeviceCsx", "DeviceCsr", "Plan", "PbError", "PHASES",
    "spgemm_symbolic", "spgemm_numeric", "spgemm_numeric_noalloc", "NOALLOC_SCRATCH_BYTES", "spgemm_plan_info", "spgemm_plan_destroy",
    "spgemm_status_string", "spgemm_last_error", "spgemm_profile_begin", "spgemm_profile_end",
    "spgemm_copy", "spgemm", "spgemm_csc", "load", "BatchPlan", "spgemm_batched_symbolic", "spgemm_batched",
    "spgemm_batch",
]


def load():
    """Load the HIP library now (raises if it is not built)."""
    return _b.lib()


def _torch():
    import torch

    return torch


@dataclasses.dataclass
class DeviceCsx:
    """A CSC or CSR matrix whose arrays are torch tensors on the GPU."""

    nrows: int
    ncols: int
    ptr: "object"  # int64 tensor
    idx: "object"  # int32 tensor
    val: "object"  # float64 tensor

    @property
    def nnz(self) -> int:
        return int(self.idx.numel())

    @classmethod
    def from_host(cls, x, device="cuda"):
        """From any object with nrows, ncols, ptr, idx, val numpy arrays."""
        torch = _torch()
        return cls(int(x.nrows), int(x.ncols),
                   torch.as_tensor(x.ptr, dtype=torch.int64).to(device),
                   torch.as_tensor(x.idx, dtype=torch.int32).to(device),
                   torch.as_tensor(x.val, dtype=torch.float64).to(device))

    def transpose_view(self) -> "DeviceCsx":
        return DeviceCsx(self.ncols, self.nrows, self.ptr, self.idx, self.val)

    def _abi(self) -> _b.PbCsx:
        torch = _torch()
        for t in (self.ptr, self.idx, self.val):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("DeviceCsx arrays must be contiguous device tensors")
        if self.ptr.dtype != torch.int64 or self.idx.dtype != torch.int32:
            raise ValueError(f"DeviceCsx needs int64 pointers and int32 indices, got {self.ptr.dtype} / {self.idx.dtype}")
        if self.val.dtype != torch.float64:
            raise ValueError(f"DeviceCsx values must be float64 (operands are double in both precisions), got "
                             f"{self.val.dtype}; an FP32c result becomes an operand with .val.double()")
        return _b.PbCsx(self.nrows, self.ncols, self.nnz, self.ptr.data_ptr(),
                        self.idx.data_ptr() if self.nnz else None, self.val.data_ptr() if self.nnz else None)


@dataclasses.dataclass
class DeviceCsr:
    """C in CSR on the GPU (colidx / val trimmed to nnz)."""

    nrows: int
    ncols: int
    rowptr: "object"
    colidx: "object"
    val: "object"

    @property
    def nnz(self) -> int:
        return int(self.colidx.numel())

    def to_host(self) -> dict:
        return dict(rowptr=self.rowptr.cpu().numpy(), colidx=self.colidx.cpu().numpy(), val=self.val.cpu().numpy())


class Plan:
    """Host-side plan from spgemm_symbolic; keeps its symbolic workspace alive."""

    def __init__(self, handle: int, sym_ws, flop: int, ws_bytes: int, precision: str):
        self.handle = ctypes.c_void_p(handle)
        self.sym_ws = sym_ws
        self.flop = flop
        self.workspace_bytes = ws_bytes
        self.precision = precision

    def info(self) -> dict:
        return spgemm_plan_info(self)

    def close(self):
        if self.handle:
            _b.lib().spgemm_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stream(stream):
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _tune(tune):
    if tune is None:
        return None
    t = _b.PbTune()
    t.tile_tuples = int(tune.get("tile_tuples", 0))
    t.expand_chunk = int(tune.get("expand_chunk", 0))
    t.round_tuples = int(tune.get("round_tuples", 0))
    t.run_align = int(tune.get("run_align", 0))
    t.row_count = int(tune.get("row_count", 0))
    t.convert = int(tune.get("convert", 0))
    t.deterministic = int(tune.get("deterministic", 0))
    return ctypes.byref(t)


def spgemm_symbolic(A: DeviceCsx, B: DeviceCsx, precision: str = "f64", tune: dict | None = None,
                    sym_ws=None, stream=None):
    """Symbolic step.  With ``sym_ws=None`` returns the symbolic workspace
    size in bytes (query mode); otherwise returns a :class:`Plan`."""
    lib = _b.lib()
    a, b = A._abi(), B._abi()
    prec = _b.PRECISIONS[precision]
    nbytes = ctypes.c_size_t(0)
    if sym_ws is None:
        _b.check(lib.spgemm_symbolic(ctypes.byref(a), ctypes.byref(b), prec, _tune(tune), None, ctypes.byref(nbytes),
                                     None, None, None, None), "spgemm_symbolic(query)")
        return int(nbytes.value)
    nbytes.value = sym_ws.numel() * sym_ws.element_size()
    plan = ctypes.c_void_p()
    flop = ctypes.c_int64()
    wsb = ctypes.c_size_t()
    _b.check(lib.spgemm_symbolic(ctypes.byref(a), ctypes.byref(b), prec, _tune(tune), sym_ws.data_ptr(),
                                 ctypes.byref(nbytes), _stream(stream), ctypes.byref(plan), ctypes.byref(flop),
                                 ctypes.byref(wsb)), "spgemm_symbolic")
    return Plan(plan.value, sym_ws, int(flop.value), int(wsb.value), precision)


def spgemm_numeric(plan: Plan, A: DeviceCsx, B: DeviceCsx, workspace, C_rowptr, C_colidx, C_val,
                   sync: bool = True, stream=None):
    """Numeric step into caller tensors.  Returns nnz(C) when ``sync``."""
    lib = _b.lib()
    a, b = A._abi(), B._abi()
    cap = int(C_colidx.numel())
    out = _b.PbCsrOut(C_rowptr.data_ptr(), C_colidx.data_ptr() if cap else None,
                      C_val.data_ptr() if cap else None, cap)
    nnz = ctypes.c_int64(-1)
    wsp = workspace.data_ptr() if workspace is not None and workspace.numel() else None
    wsb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _b.check(lib.spgemm_numeric(plan.handle, ctypes.byref(a), ctypes.byref(b), wsp, wsb, ctypes.byref(out),
                                ctypes.byref(nnz) if sync else None, _stream(stream)), "spgemm_numeric")
    return int(nnz.value) if sync else None


def spgemm_numeric_noalloc(plan: Plan, A: DeviceCsx, B: DeviceCsx, C_rowptr, C_colidx, C_val,
                           sync: bool = True, stream=None):
    """Numeric step into caller tensors with no workspace argument: the
    library's own per-GPU device scratch of NOALLOC_SCRATCH_BYTES holds the
    workspace, and nothing is allocated.  Returns nnz(C) when ``sync``."""
    lib = _b.lib()
    a, b = A._abi(), B._abi()
    cap = int(C_colidx.numel())
    out = _b.PbCsrOut(C_rowptr.data_ptr(), C_colidx.data_ptr() if cap else None,
                      C_val.data_ptr() if cap else None, cap)
    nnz = ctypes.c_int64(-1)
    _b.check(lib.spgemm_numeric_noalloc(plan.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(out),
                                        ctypes.byref(nnz) if sync else None, _stream(stream)),
             "spgemm_numeric_noalloc")
    return int(nnz.value) if sync else None


def spgemm_plan_rounds(plan: Plan):
    """(row_begin, flop_per_round): round r computes rows
    [row_begin[r], row_begin[r+1]) of C and expands flop_per_round[r] tuples."""
    lib = _b.lib()
    n = ctypes.c_int64(0)
    _b.check(lib.spgemm_plan_rounds(plan.handle, ctypes.byref(n), None, None), "spgemm_plan_rounds")
    rb = (ctypes.c_int64 * (n.value + 1))()
    fl = (ctypes.c_int64 * max(n.value, 1))()
    _b.check(lib.spgemm_plan_rounds(plan.handle, ctypes.byref(n), rb, fl), "spgemm_plan_rounds")
    return [int(x) for x in rb], [int(fl[i]) for i in range(n.value)]


def spgemm_numeric_round(plan: Plan, A: DeviceCsx, B: DeviceCsx, round_index: int, workspace, C_rowptr, C_colidx,
                         C_val, sync: bool = True, stream=None):
    """Rows of one round of C into caller tensors (row pointers start at 0).
    Returns the round's nnz when ``sync``."""
    lib = _b.lib()
    a, b = A._abi(), B._abi()
    cap = int(C_colidx.numel())
    out = _b.PbCsrOut(C_rowptr.data_ptr(), C_colidx.data_ptr() if cap else None,
                      C_val.data_ptr() if cap else None, cap)
    nnz = ctypes.c_int64(-1)
    wsp = workspace.data_ptr() if workspace is not None and workspace.numel() else None
    wsb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _b.check(lib.spgemm_numeric_round(plan.handle, ctypes.byref(a), ctypes.byref(b), int(round_index), wsp, wsb,
                                      ctypes.byref(out), ctypes.byref(nnz) if sync else None, _stream(stream)),
             "spgemm_numeric_round")
    return int(nnz.value) if sync else None


def spgemm_plan_info(plan: Plan) -> dict:
    info = _b.PbPlanInfo()
    _b.check(_b.lib().spgemm_plan_info(plan.handle, ctypes.byref(info)), "spgemm_plan_info")
    return {name: getattr(info, name) for name, _ in _b.PbPlanInfo._fields_}


def spgemm_plan_destroy(plan: Plan) -> None:
    plan.close()


def spgemm_status_string(status: int) -> str:
    return _b.status_string(status)


def spgemm_last_error() -> str:
    return _b.last_error()


def spgemm_profile_begin() -> None:
    _b.check(_b.lib().spgemm_profile_begin(), "spgemm_profile_begin")


def spgemm_profile_end() -> dict:
    prof = _b.PbProfile()
    _b.check(_b.lib().spgemm_profile_end(ctypes.byref(prof)), "spgemm_profile_end")
    return {name: (prof.ms[i], prof.launches[i]) for i, name in enumerate(PHASES)}


def spgemm_copy(dst, src, nbytes: int, stream=None) -> None:
    _b.check(_b.lib().spgemm_copy(dst.data_ptr(), src.data_ptr(), int(nbytes), _stream(stream)), "spgemm_copy")


def _alloc_bytes(n: int, device):
    torch = _torch()
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


def spgemm(A: DeviceCsx, B: DeviceCsx, precision: str = "f64", tune: dict | None = None, stream=None) -> DeviceCsr:
    """C = A*B (A CSC, B CSR) on the GPU; allocation through torch."""
    torch = _torch()
    dev = A.ptr.device
    nsym = spgemm_symbolic(A, B, precision, tune)
    sym_ws = _alloc_bytes(nsym, dev)
    plan = spgemm_symbolic(A, B, precision, tune, sym_ws=sym_ws, stream=stream)
    try:
        ws = _alloc_bytes(plan.workspace_bytes, dev)
        rowptr = torch.empty(A.nrows + 1, dtype=torch.int64, device=dev)
        cap = max(plan.flop, 1)
        colidx = torch.empty(cap, dtype=torch.int32, device=dev)
        val = torch.empty(cap, dtype=torch.float64 if precision == "f64" else torch.float32, device=dev)
        nnz = spgemm_numeric(plan, A, B, ws, rowptr, colidx, val, sync=True, stream=stream)
    finally:
        plan.close()
    return DeviceCsr(A.nrows, B.ncols, rowptr, colidx[:nnz], val[:nnz])


def spgemm_csc(A: DeviceCsx, B: DeviceCsx, precision: str = "f64", tune: dict | None = None,
               stream=None) -> DeviceCsx:
    """C = A*B returned in CSC (A CSC, B CSR), with no extra pass: C in CSC
    has the arrays of C^T = B^T * A^T in CSR, and B^T in CSC (A^T in CSR)
    are B's (A's) own arrays read the other way round.  With "f32c" the
    values are float32; to use the result as an operand, convert them
    (``DeviceCsx(c.nrows, c.ncols, c.ptr, c.idx, c.val.double())``)."""
    ct = spgemm(B.transpose_view(), A.transpose_view(), precision=precision, tune=tune, stream=stream)
    return DeviceCsx(A.nrows, B.ncols, ct.rowptr, ct.colidx, ct.val)


# ---------------------------------------------------------------- batches
class BatchPlan(Plan):
    """Plan of a batch; ``flops[i]`` is problem i's multiplication count."""

    def __init__(self, handle: int, sym_ws, flops, ws_bytes: int, precision: str):
        super().__init__(handle, sym_ws, int(sum(flops)), ws_bytes, precision)
        self.flops = list(flops)
        self.count = len(self.flops)


def _abi_array(mats):
    arr = (_b.PbCsx * len(mats))()
    for i, x in enumerate(mats):
        arr[i] = x._abi()
    return arr


def spgemm_batched_symbolic(pairs, precision: str = "f64", tune: dict | None = None, sym_ws=None, stream=None):
    """Symbolic step for a batch of (A_csc, B_csr) pairs.  With
    ``sym_ws=None`` returns the workspace size (query); else a BatchPlan."""
    lib = _b.lib()
    count = len(pairs)
    aa = _abi_array([a for a, _ in pairs])
    bb = _abi_array([b for _, b in pairs])
    prec = _b.PRECISIONS[precision]
    nbytes = ctypes.c_size_t(0)
    if sym_ws is None:
        _b.check(lib.spgemm_batched_symbolic(count, aa, bb, prec, _tune(tune), None, ctypes.byref(nbytes), None, None,
                                             None, None), "spgemm_batched_symbolic(query)")
        return int(nbytes.value)
    nbytes.value = sym_ws.numel() * sym_ws.element_size()
    plan = ctypes.c_void_p()
    flops = (ctypes.c_int64 * count)()
    wsb = ctypes.c_size_t()
    _b.check(lib.spgemm_batched_symbolic(count, aa, bb, prec, _tune(tune), sym_ws.data_ptr(), ctypes.byref(nbytes),
                                         _stream(stream), ctypes.byref(plan), flops, ctypes.byref(wsb)),
             "spgemm_batched_symbolic")
    return BatchPlan(plan.value, sym_ws, [int(f) for f in flops], int(wsb.value), precision)


def spgemm_batched(plan: BatchPlan, pairs, workspace, outs, sync: bool = True, stream=None):
    """Numeric step for the whole batch.  ``outs[i] = (rowptr, colidx, val)``
    device tensors.  Returns the list of nnz(C_i) when ``sync``; with
    ``sync=False`` only enqueues work (capturable in a HIP graph)."""
    lib = _b.lib()
    count = len(pairs)
    aa = _abi_array([a for a, _ in pairs])
    bb = _abi_array([b for _, b in pairs])
    cc = (_b.PbCsrOut * count)()
    for i, (rp, ci, cv) in enumerate(outs):
        cap = int(ci.numel())
        cc[i] = _b.PbCsrOut(rp.data_ptr(), ci.data_ptr() if cap else None, cv.data_ptr() if cap else None, cap)
    nnz = (ctypes.c_int64 * count)()
    wsp = workspace.data_ptr() if workspace is not None and workspace.numel() else None
    wsb = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _b.check(lib.spgemm_batched(plan.handle, count, aa, bb, wsp, wsb, cc, nnz if sync else None, _stream(stream)),
             "spgemm_batched")
    return [int(x) for x in nnz] if sync else None


def spgemm_batch(pairs, precision: str = "f64", tune: dict | None = None, stream=None):
    """C_i = A_i * B_i for a list of (A_csc, B_csr) pairs, as one batch."""
    torch = _torch()
    dev = pairs[0][0].ptr.device
    nsym = spgemm_batched_symbolic(pairs, precision, tune)
    plan = spgemm_batched_symbolic(pairs, precision, tune, sym_ws=_alloc_bytes(nsym, dev), stream=stream)
    try:
        ws = _alloc_bytes(plan.workspace_bytes, dev)
        vdt = torch.float64 if precision == "f64" else torch.float32
        outs = [(torch.empty(a.nrows + 1, dtype=torch.int64, device=dev),
                 torch.empty(max(f, 1), dtype=torch.int32, device=dev),
                 torch.empty(max(f, 1), dtype=vdt, device=dev)) for (a, _), f in zip(pairs, plan.flops)]
        nnz = spgemm_batched(plan, pairs, ws, outs, sync=True, stream=stream)
    finally:
        plan.close()
    return [DeviceCsr(a.nrows, b.ncols, rp, ci[:z], cv[:z]) for (a, b), (rp, ci, cv), z in zip(pairs, outs, nnz)]
