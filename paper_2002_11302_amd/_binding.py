"""ctypes marshalling for libpbspgemm.so (declarations in include/pbspgemm.h).

Argument marshalling only: every step of the product runs in the HIP
library.  If the library is missing this module raises; there is no other
implementation to fall back on.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# PB_LIB names another build of the same library (the sanitizer test's host
# build); there is no other implementation to fall back to.
LIB_PATH = os.environ.get("PB_LIB") or os.path.join(_PKG, "libpbspgemm.so")

PB_OK = 0
STATUS_NAMES = {
    0: "PB_OK", 1: "PB_ERR_ARG", 2: "PB_ERR_SHAPE", 3: "PB_ERR_RANGE", 4: "PB_ERR_WORKSPACE",
    5: "PB_ERR_CAPACITY", 6: "PB_ERR_HIP", 7: "PB_ERR_UNSUPPORTED", 8: "PB_ERR_INTERNAL",
}
PRECISIONS = {"f64": 0, "f32c": 1}
PB_NPHASES = 5
PHASES = ("symbolic", "expand", "sort_compress", "row_counts", "wide_partition")
NOALLOC_SCRATCH_BYTES = 64 << 20  # PB_NOALLOC_SCRATCH_BYTES


class PbError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {detail}")


class PbCsx(ctypes.Structure):
    _fields_ = [
        ("nrows", ctypes.c_int64), ("ncols", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("ptr", ctypes.c_void_p), ("idx", ctypes.c_void_p), ("val", ctypes.c_void_p),
    ]


class PbCsrOut(ctypes.Structure):
    _fields_ = [("rowptr", ctypes.c_void_p), ("colidx", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("capacity", ctypes.c_int64)]


class PbTune(ctypes.Structure):
    _fields_ = [("tile_tuples", ctypes.c_int32), ("expand_chunk", ctypes.c_int32), ("round_tuples", ctypes.c_int64),
                ("run_align", ctypes.c_int32), ("row_count", ctypes.c_int32),
                ("convert", ctypes.c_int32), ("deterministic", ctypes.c_int32)]


class PbPlanInfo(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("k", ctypes.c_int64), ("n", ctypes.c_int64), ("flop", ctypes.c_int64),
        ("nbins", ctypes.c_int64), ("max_bin_tuples", ctypes.c_int64), ("max_row_flop", ctypes.c_int64),
        ("tile_tuples", ctypes.c_int32), ("expand_chunk", ctypes.c_int32), ("col_bits", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("count", ctypes.c_int64), ("slots", ctypes.c_int64),
        ("run_align", ctypes.c_int32), ("row_count", ctypes.c_int32),
        ("deterministic", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class PbProfile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * PB_NPHASES), ("launches", ctypes.c_int64 * PB_NPHASES)]


_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i64 = ctypes.c_int64

# name -> (restype, argtypes)
SIGNATURES = {
    "spgemm_symbolic": (ctypes.c_int, [ctypes.POINTER(PbCsx), ctypes.POINTER(PbCsx), ctypes.c_int, ctypes.POINTER(PbTune),
                                       _vp, ctypes.POINTER(_sz), _vp, ctypes.POINTER(_vp), ctypes.POINTER(_i64),
                                       ctypes.POINTER(_sz)]),
    "spgemm_numeric": (ctypes.c_int, [_vp, ctypes.POINTER(PbCsx), ctypes.POINTER(PbCsx), _vp, _sz,
                                      ctypes.POINTER(PbCsrOut), ctypes.POINTER(_i64), _vp]),
    "spgemm_numeric_noalloc": (ctypes.c_int, [_vp, ctypes.POINTER(PbCsx), ctypes.POINTER(PbCsx),
                                              ctypes.POINTER(PbCsrOut), ctypes.POINTER(_i64), _vp]),
    "spgemm_plan_info": (ctypes.c_int, [_vp, ctypes.POINTER(PbPlanInfo)]),
    "spgemm_plan_rounds": (ctypes.c_int, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "spgemm_numeric_round": (ctypes.c_int, [_vp, ctypes.POINTER(PbCsx), ctypes.POINTER(PbCsx), _i64, _vp, _sz,
                                            ctypes.POINTER(PbCsrOut), ctypes.POINTER(_i64), _vp]),
    "spgemm_plan_destroy": (None, [_vp]),
    "spgemm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "spgemm_last_error": (ctypes.c_char_p, []),
    "spgemm_profile_begin": (ctypes.c_int, []),
    "spgemm_profile_end": (ctypes.c_int, [ctypes.POINTER(PbProfile)]),
    "spgemm_copy": (ctypes.c_int, [_vp, _vp, _sz, _vp]),
    "spgemm_batched_symbolic": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(PbCsx), ctypes.POINTER(PbCsx), ctypes.c_int,
                                               ctypes.POINTER(PbTune), _vp, ctypes.POINTER(_sz), _vp, ctypes.POINTER(_vp),
                                               ctypes.POINTER(_i64), ctypes.POINTER(_sz)]),
    "spgemm_batched": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(PbCsx), ctypes.POINTER(PbCsx), _vp, _sz,
                                      ctypes.POINTER(PbCsrOut), ctypes.POINTER(_i64), _vp]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2002_11302_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status: int, where: str) -> None:
    if status != PB_OK:
        detail = lib().spgemm_last_error().decode(errors="replace")
        raise PbError(status, where, detail)


def last_error() -> str:
    return lib().spgemm_last_error().decode(errors="replace")


def status_string(status: int) -> str:
    return lib().spgemm_status_string(int(status)).decode()
