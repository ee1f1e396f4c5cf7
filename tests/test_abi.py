"""C-ABI checks that need no GPU: the library loads, exports every entry
point the header declares, and rejects bad arguments on the host before any
device work."""
import ctypes
import os
import re

import pytest

from paper_2002_11302_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pbspgemm.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^(?:const\s+)?\w+\s*\*?\s*(spgemm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        from paper_2002_11302_amd import build

        build.build()
    return B.lib()


def test_header_symbols_exported(lib):
    names = _declared_functions()
    assert len(names) >= 9, names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in the header but not exported"
        assert n in B.SIGNATURES, f"{n} has no binding"


def test_status_strings(lib):
    for code, name in B.STATUS_NAMES.items():
        assert B.status_string(code) == name


def _fake(nrows, ncols, nnz, ptr=0x1000, idx=0x2000, val=0x3000):
    return B.PbCsx(nrows, ncols, nnz, ptr, idx, val)


def _symbolic(lib, a, b, prec=0, tune=None, ws=None, nbytes=0):
    sz = ctypes.c_size_t(nbytes)
    plan = ctypes.c_void_p()
    flop = ctypes.c_int64()
    wsb = ctypes.c_size_t()
    rc = lib.spgemm_symbolic(ctypes.byref(a), ctypes.byref(b), prec, tune, ws, ctypes.byref(sz), None,
                             ctypes.byref(plan), ctypes.byref(flop), ctypes.byref(wsb))
    return rc, sz.value


def test_query_mode_sizes(lib):
    rc, n1 = _symbolic(lib, _fake(1000, 500, 10), _fake(500, 700, 10))
    assert rc == 0 and n1 > 0
    rc, n2 = _symbolic(lib, _fake(2000, 500, 10), _fake(500, 700, 10))
    assert rc == 0 and n2 > n1  # grows with the row count


def test_shape_mismatch(lib):
    rc, _ = _symbolic(lib, _fake(10, 5, 3), _fake(6, 7, 3))
    assert B.STATUS_NAMES[rc] == "PB_ERR_SHAPE"
    assert "A.ncols" in B.last_error()


def test_negative_and_range(lib):
    rc, _ = _symbolic(lib, _fake(-1, 5, 0), _fake(5, 7, 0))
    assert B.STATUS_NAMES[rc] == "PB_ERR_SHAPE"
    rc, _ = _symbolic(lib, _fake(1 << 31, 5, 0), _fake(5, 7, 0))
    assert B.STATUS_NAMES[rc] == "PB_ERR_RANGE"
    rc, _ = _symbolic(lib, _fake(10, 5, 0), _fake(5, 1 << 31, 0))
    assert B.STATUS_NAMES[rc] == "PB_ERR_RANGE"


def test_null_pointers(lib):
    rc, _ = _symbolic(lib, _fake(10, 5, 3, ptr=None), _fake(5, 7, 3))
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"
    rc, _ = _symbolic(lib, _fake(10, 5, 3), _fake(5, 7, 3, idx=None))
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"
    # empty matrices may have null idx / val
    rc, _ = _symbolic(lib, _fake(10, 5, 0, idx=None, val=None), _fake(5, 7, 0, idx=None, val=None))
    assert rc == 0


def test_bad_precision_and_tune(lib):
    rc, _ = _symbolic(lib, _fake(10, 5, 3), _fake(5, 7, 3), prec=7)
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"
    t = B.PbTune()
    t.tile_tuples = 100
    rc, _ = _symbolic(lib, _fake(10, 5, 3), _fake(5, 7, 3), tune=ctypes.byref(t))
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"
    t = B.PbTune()
    t.expand_chunk = 1000
    rc, _ = _symbolic(lib, _fake(10, 5, 3), _fake(5, 7, 3), tune=ctypes.byref(t))
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"
    t = B.PbTune()
    t.round_tuples = -1
    rc, _ = _symbolic(lib, _fake(10, 5, 3), _fake(5, 7, 3), tune=ctypes.byref(t))
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"


def test_tune_struct_layout():
    """pb_tune is 32 bytes with round_tuples at offset 8 and run_align at 16
    (as in the header)."""
    assert ctypes.sizeof(B.PbTune) == 32
    assert B.PbTune.round_tuples.offset == 8
    assert B.PbTune.run_align.offset == 16
    assert B.PbTune.row_count.offset == 20
    assert B.PbTune.convert.offset == 24
    assert B.PbTune.deterministic.offset == 28
    assert ctypes.sizeof(B.PbPlanInfo) % 8 == 0
    assert B.PbPlanInfo.deterministic.offset == B.PbPlanInfo.row_count.offset + 4


def test_deterministic_tune_checks(lib):
    """The fixed summation order takes 0/1, needs row buckets and the
    count-pass ConvertCSR; its symbolic workspace adds four 32-bit words
    per entry of A (record entry, and the per-row grouped lists)."""
    a, b = _fake(1000, 500, 3000), _fake(500, 700, 3000)
    for field, value in (("deterministic", 2), ("deterministic", -1)):
        t = B.PbTune()
        setattr(t, field, value)
        rc, _ = _symbolic(lib, a, b, tune=ctypes.byref(t))
        assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"
    for field, value in (("convert", 2), ("row_count", 1)):
        t = B.PbTune()
        t.deterministic = 1
        setattr(t, field, value)
        rc, _ = _symbolic(lib, a, b, tune=ctypes.byref(t))
        assert B.STATUS_NAMES[rc] == "PB_ERR_ARG", field
    t = B.PbTune()
    t.deterministic = 1
    t.convert = 1
    rc, det = _symbolic(lib, a, b, tune=ctypes.byref(t))
    assert rc == 0
    rc, plain = _symbolic(lib, a, b)
    assert rc == 0 and det >= plain + 16 * 3000
    # too many rows for row buckets: no fixed order
    t = B.PbTune()
    t.deterministic = 1
    rc, _ = _symbolic(lib, _fake((1 << 25) + 1, 5, 3), _fake(5, 7, 3), tune=ctypes.byref(t))
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"


def test_bad_row_count(lib):
    t = B.PbTune()
    t.row_count = 3
    rc, _ = _symbolic(lib, _fake(10, 5, 3), _fake(5, 7, 3), tune=ctypes.byref(t))
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"
    # row buckets need at most 2^25 rows
    t.row_count = 2
    rc, _ = _symbolic(lib, _fake((1 << 25) + 1, 5, 3), _fake(5, 7, 3), tune=ctypes.byref(t))
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"


def test_row_bucket_workspace(lib):
    """The row-bucket symbolic step needs its histogram and entry records in
    the symbolic workspace (8 bytes per entry of A on top of the atomic form)."""
    sizes = {}
    for mode in (1, 2):
        t = B.PbTune()
        t.row_count = mode
        rc, need = _symbolic(lib, _fake(1000, 500, 3000), _fake(500, 700, 3000), tune=ctypes.byref(t))
        assert rc == 0
        sizes[mode] = need
    assert sizes[2] >= sizes[1] + 8 * 3000
    rc, auto = _symbolic(lib, _fake(1000, 500, 3000), _fake(500, 700, 3000))
    assert rc == 0 and auto == sizes[2]


def test_bad_run_align(lib):
    t = B.PbTune()
    t.run_align = 3
    rc, _ = _symbolic(lib, _fake(10, 5, 3), _fake(5, 7, 3), tune=ctypes.byref(t))
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"


def test_symbolic_workspace_too_small(lib):
    rc, need = _symbolic(lib, _fake(100, 50, 3), _fake(50, 70, 3))
    assert rc == 0
    rc, _ = _symbolic(lib, _fake(100, 50, 3), _fake(50, 70, 3), ws=0x10000, nbytes=need - 1)
    assert B.STATUS_NAMES[rc] == "PB_ERR_WORKSPACE"


def test_numeric_null_plan(lib):
    a, b = _fake(10, 5, 3), _fake(5, 7, 3)
    out = B.PbCsrOut(0x1000, 0x2000, 0x3000, 10)
    rc = lib.spgemm_numeric(None, ctypes.byref(a), ctypes.byref(b), None, 0, ctypes.byref(out), None, None)
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"


def test_rounds_null_plan(lib):
    n = ctypes.c_int64(0)
    assert B.STATUS_NAMES[lib.spgemm_plan_rounds(None, ctypes.byref(n), None, None)] == "PB_ERR_ARG"
    a, b = _fake(10, 5, 3), _fake(5, 7, 3)
    out = B.PbCsrOut(0x1000, 0x2000, 0x3000, 10)
    rc = lib.spgemm_numeric_round(None, ctypes.byref(a), ctypes.byref(b), 0, None, 0, ctypes.byref(out), None, None)
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"


def test_copy_alignment(lib):
    rc = lib.spgemm_copy(0x1001, 0x2000, 64, None)
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"
    rc = lib.spgemm_copy(0x1000, 0x2000, 63, None)
    assert B.STATUS_NAMES[rc] == "PB_ERR_ARG"


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        B.lib()


def test_env_tune_fills_unset_fields(lib, monkeypatch):
    """PB_TUNE fills the tuning fields a call leaves at 0: row_count=1
    (device atomics) changes the symbolic workspace size, an explicit
    row_count in the call wins over it, and a malformed value or an unknown
    key is PB_ERR_ARG."""
    a, b = _fake(1000, 500, 3000), _fake(500, 700, 3000)
    rc, auto = _symbolic(lib, a, b)
    assert rc == 0
    t1 = B.PbTune()
    t1.row_count = 1
    rc, atomics = _symbolic(lib, a, b, tune=ctypes.byref(t1))
    assert rc == 0 and atomics != auto
    monkeypatch.setenv("PB_TUNE", " row_count = 1 ; tile_tuples=4096")
    assert _symbolic(lib, a, b) == (0, atomics)
    t2 = B.PbTune()
    t2.row_count = 2
    assert _symbolic(lib, a, b, tune=ctypes.byref(t2)) == (0, auto)
    for bad in ("row_count", "row_count=x", "bogus=1", "tile_tuples=100", "deterministic=1,row_count=1"):
        monkeypatch.setenv("PB_TUNE", bad)
        rc, _ = _symbolic(lib, a, b)
        assert B.STATUS_NAMES[rc] == "PB_ERR_ARG", bad
    monkeypatch.setenv("PB_TUNE", "")
    assert _symbolic(lib, a, b) == (0, auto)
