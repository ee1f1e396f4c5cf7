"""CPU oracle for sparse C = A*B -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path never does,
and this package imports nothing from the product.

The arithmetic lives in ``spgemm_oracle.c`` (plain C, double precision,
``-ffp-contract=off``): Gustavson's column-by-column product with a sorted
accumulator (paper Section 2.2, Fig. 1), each output C(r,j) being the sum of
the rounded products A(r,k)*B(k,j) over ascending k, added one at a time.
Merging keeps every position that receives a tuple, so cancelled sums stay
stored (paper Section 2.2: C is C^ with equal (row, col) tuples added).

Functions here only marshal arrays and call the C routines:

* :func:`flop` -- the symbolic multiplication count of Algorithm 3.
* :func:`spgemm` -- all of C in CSR, plus N = |A||B| per stored entry.
* :func:`spgemm_rows` -- selected rows of C, through the identity
  (A B)^T = B^T A^T: the CSR arrays of B are the CSC arrays of B^T and the
  CSC arrays of A are the CSR arrays of A^T, so rows of C are columns of
  B^T A^T, computed by the same column routine with the same ascending-k
  summation order.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spgemm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU code, no shared sources)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        path = os.environ.get("PB_ORACLE_LIB")  # another build of the same source (the sanitizer test)
        if not path:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            path = _LIB
        lib = ctypes.CDLL(path)
        lib.oracle_flop.restype = ctypes.c_int64
        lib.oracle_flop.argtypes = [ctypes.c_int64, _i64p, _i64p]
        lib.oracle_spgemm_cols.restype = ctypes.c_int
        lib.oracle_spgemm_cols.argtypes = [
            ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            _i64p, _i32p, _f64p, _i64p, _i32p, _f64p,
            ctypes.c_int64, _i64p, ctypes.c_int,
            ctypes.POINTER(_i64p), ctypes.POINTER(_i32p), ctypes.POINTER(_f64p), ctypes.POINTER(_f64p),
        ]
        lib.oracle_transpose.restype = ctypes.c_int
        lib.oracle_transpose.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _f64p, _i64p, _i32p, _f64p]
        lib.oracle_free.argtypes = [ctypes.c_void_p]
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _cf(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def flop(a_colptr, b_rowptr) -> int:
    """Algorithm 3: sum over k of nnz(A(:,k)) * nnz(B(k,:))."""
    a_colptr = _c64(a_colptr)
    b_rowptr = _c64(b_rowptr)
    assert a_colptr.size == b_rowptr.size
    return int(_load().oracle_flop(a_colptr.size - 1, _p(a_colptr, _i64p), _p(b_rowptr, _i64p)))


def _cols(m, k, n, a_ptr, a_idx, a_val, b_ptr, b_idx, b_val, cols, nthreads):
    lib = _load()
    a_ptr, a_idx, a_val = _c64(a_ptr), _c32(a_idx), _cf(a_val)
    b_ptr, b_idx, b_val = _c64(b_ptr), _c32(b_idx), _cf(b_val)
    assert a_ptr.size == k + 1 and b_ptr.size == k + 1
    if cols is None:
        nsel, cptr = n, None
    else:
        cols = _c64(cols)
        nsel, cptr = cols.size, _p(cols, _i64p)
    op, oi, ov, oa = _i64p(), _i32p(), _f64p(), _f64p()
    rc = lib.oracle_spgemm_cols(
        m, k, n, _p(a_ptr, _i64p), _p(a_idx, _i32p), _p(a_val, _f64p),
        _p(b_ptr, _i64p), _p(b_idx, _i32p), _p(b_val, _f64p),
        nsel, cptr, int(nthreads), ctypes.byref(op), ctypes.byref(oi), ctypes.byref(ov), ctypes.byref(oa))
    if rc != 0:
        raise MemoryError("oracle_spgemm_cols failed")
    try:
        ptr = np.ctypeslib.as_array(op, shape=(nsel + 1,)).copy()
        tot = int(ptr[-1])
        idx = np.ctypeslib.as_array(oi, shape=(max(tot, 1),))[:tot].copy()
        val = np.ctypeslib.as_array(ov, shape=(max(tot, 1),))[:tot].copy()
        abv = np.ctypeslib.as_array(oa, shape=(max(tot, 1),))[:tot].copy()
    finally:
        for q in (op, oi, ov, oa):
            lib.oracle_free(ctypes.cast(q, ctypes.c_void_p))
    return ptr, idx, val, abv


def transpose(nmajor, nminor, ptr, idx, val):
    """Stable counting-sort transpose of compressed storage (C routine)."""
    lib = _load()
    ptr, idx = _c64(ptr), _c32(idx)
    val = None if val is None else _cf(val)
    nnz = int(ptr[-1])
    tptr = np.zeros(nminor + 1, np.int64)
    tidx = np.zeros(max(nnz, 1), np.int32)
    tval = np.zeros(max(nnz, 1), np.float64)
    rc = lib.oracle_transpose(nmajor, nminor, _p(ptr, _i64p), _p(idx, _i32p),
                              None if val is None else _p(val, _f64p),
                              _p(tptr, _i64p), _p(tidx, _i32p), _p(tval, _f64p))
    if rc != 0:
        raise MemoryError("oracle_transpose failed")
    return tptr, tidx[:nnz], (None if val is None else tval[:nnz])


def spgemm(a_csc, b_csr, nthreads: int = 0) -> dict:
    """All of C = A*B.  ``a_csc``/``b_csr`` expose nrows, ncols, ptr, idx, val.

    Returns dict(rowptr, colidx, val, absval, flop, nrows, ncols) with C in
    CSR (columns ascending in each row); ``absval`` is N = |A||B| per entry.
    """
    m, k, n = a_csc.nrows, a_csc.ncols, b_csr.ncols
    assert b_csr.nrows == k
    cptr, cidx, cval, cabs = _cols(m, k, n, a_csc.ptr, a_csc.idx, a_csc.val,
                                   b_csr.ptr, b_csr.idx, b_csr.val, None, nthreads)
    # CSC -> CSR by a stable counting sort; rows then hold ascending columns.
    rptr, ridx, rval = transpose(n, m, cptr, cidx, cval)
    _, _, rabs = transpose(n, m, cptr, cidx, cabs)
    return dict(rowptr=rptr, colidx=ridx, val=rval, absval=rabs,
                flop=flop(a_csc.ptr, b_csr.ptr), nrows=m, ncols=n)


def spgemm_cols(a_csc, b_csr, cols, nthreads: int = 0) -> dict:
    """Selected columns of C (CSC pieces in the order of ``cols``)."""
    m, k, n = a_csc.nrows, a_csc.ncols, b_csr.ncols
    ptr, idx, val, abv = _cols(m, k, n, a_csc.ptr, a_csc.idx, a_csc.val,
                               b_csr.ptr, b_csr.idx, b_csr.val, cols, nthreads)
    return dict(ptr=ptr, idx=idx, val=val, absval=abv)


def spgemm_rows(a_csc, b_csr, rows, nthreads: int = 0) -> dict:
    """Selected rows of C via C^T = B^T A^T (see module docstring).

    Returns dict(ptr, idx, val, absval): row ``rows[s]`` of C occupies
    ``idx[ptr[s]:ptr[s+1]]`` with columns ascending.
    """
    m, k, n = a_csc.nrows, a_csc.ncols, b_csr.ncols
    # B^T: n x k, its CSC arrays are B's CSR arrays; A^T: k x m, its CSR
    # arrays are A's CSC arrays.
    ptr, idx, val, abv = _cols(n, k, m, b_csr.ptr, b_csr.idx, b_csr.val,
                               a_csc.ptr, a_csc.idx, a_csc.val, rows, nthreads)
    return dict(ptr=ptr, idx=idx, val=val, absval=abv)
