"""The opt-in content check of the operands (PB_VALIDATE=1): the symbolic
step copies each operand's pointer and index arrays to the host and rejects
a malformed matrix with PB_ERR_ARG before any kernel is launched, so these
malformed inputs never reach the GPU kernels."""
import sys

import numpy as np
import pytest

import oracle
from workloads import Csx, er_problem

pytestmark = pytest.mark.gpu


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


@pytest.fixture()
def validate(monkeypatch):
    monkeypatch.setenv("PB_VALIDATE", "1")


def _copy(x: Csx, **kw) -> Csx:
    return Csx(x.nrows, x.ncols, kw.get("ptr", x.ptr.copy()), kw.get("idx", x.idx.copy()),
               kw.get("val", x.val.copy()), x.fmt)


def _line_with(x: Csx, n: int) -> int:
    """First line (column of a CSC, row of a CSR) with at least n entries."""
    return int(np.nonzero(np.diff(x.ptr) >= n)[0][0])


def test_valid_input_same_result(pb, validate):
    _say("PB_VALIDATE=1 on a valid ER product")
    a, b = er_problem(512, 6, 11, 12)
    got = pb.spgemm(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b)).to_host()
    ref = oracle.spgemm(a, b)
    assert np.array_equal(got["rowptr"], ref["rowptr"]) and np.array_equal(got["colidx"], ref["colidx"])
    assert np.all(np.abs(got["val"] - ref["val"]) <= 1e-12 * ref["absval"])


def _bad_cases():
    a, b = er_problem(256, 4, 21, 22)
    cases = []
    j = _line_with(a, 2)
    idx = a.idx.copy()
    idx[a.ptr[j]], idx[a.ptr[j] + 1] = idx[a.ptr[j] + 1], idx[a.ptr[j]]
    cases.append(("A indices out of order", _copy(a, idx=idx), b, "strictly increasing"))
    idx = a.idx.copy()
    idx[a.ptr[j] + 1] = idx[a.ptr[j]]
    cases.append(("A repeated index", _copy(a, idx=idx), b, "strictly increasing"))
    idx = a.idx.copy()
    idx[a.ptr[j + 1] - 1] = a.nrows
    cases.append(("A row index = m", _copy(a, idx=idx), b, "out of"))
    idx = a.idx.copy()
    idx[a.ptr[j]] = -1
    cases.append(("A negative row index", _copy(a, idx=idx), b, "out of"))
    ptr = b.ptr.copy()
    r = b.nrows // 2
    assert ptr[r] > 0
    ptr[r + 1] = ptr[r] - 1
    cases.append(("B pointers decrease", a, _copy(b, ptr=ptr), "ptr decreases"))
    ptr = b.ptr.copy()
    ptr[-1] -= 1
    cases.append(("B ptr[end] != nnz", a, _copy(b, ptr=ptr), "not nnz"))
    ptr = b.ptr.copy()
    ptr[0] = 1
    cases.append(("B ptr[0] != 0", a, _copy(b, ptr=ptr), "ptr[0]"))
    return cases


@pytest.mark.parametrize("case", range(7))
def test_malformed_operand_rejected(pb, validate, case):
    name, a, b, text = _bad_cases()[case]
    _say(f"PB_VALIDATE=1: {name}")
    with pytest.raises(pb.PbError) as ei:
        pb.spgemm(pb.DeviceCsx.from_host(a), pb.DeviceCsx.from_host(b))
    assert ei.value.name == "PB_ERR_ARG" and text in str(ei.value)


def test_malformed_batch_member_rejected(pb, validate):
    _say("PB_VALIDATE=1: batch with one malformed member")
    good = [er_problem(128, 3, 31 + i, 41 + i) for i in range(3)]
    name, bad_a, bad_b, text = _bad_cases()[2]
    pairs = [(pb.DeviceCsx.from_host(x), pb.DeviceCsx.from_host(y)) for x, y in good]
    pairs.insert(1, (pb.DeviceCsx.from_host(bad_a), pb.DeviceCsx.from_host(bad_b)))
    with pytest.raises(pb.PbError) as ei:
        pb.spgemm_batch(pairs)
    assert ei.value.name == "PB_ERR_ARG" and "A[1]" in str(ei.value)
