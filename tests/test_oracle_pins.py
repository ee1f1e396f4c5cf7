"""Pins for the CPU oracle, each independent of the oracle's own code.

The oracle computes C = A*B (paper Section 2.1): C(i,j) is the sum over k of
A(i,k)*B(k,j), and a position is stored when at least one product lands on
it (merging adds tuples with equal row and column, Section 2.2), so
cancelled sums stay stored.  The pins below fix that definition from
outside the oracle:

* hand-worked examples stored under tests/golden/ (a 3x3 product and a
  cancellation, integer arithmetic done by hand);
* brute force by pure-Python loops in ascending k on tiny random inputs,
  including empty / full rows and columns, rectangular shapes, stored zeros
  and cancellation (structure and bit-exact values);
* exact special cases: integer-valued inputs against numpy's dense product,
  A*I = A, I*B = B, permutations and diagonal scalings;
* the transpose identity (AB)^T = B^T A^T, bit for bit;
* Algorithm 3's flop count against the ER closed form d^2 n, and the bound
  nnz(C) <= flop that follows from cf >= 1 (Section 2.1);
* scipy's sparse product (an independent library routine) on positive
  inputs, where no sum cancels;
* mutation checks: plausible mistakes planted in a copy of the oracle's
  output (a dropped term, a flipped sign, a transposed operand, a lost
  structural zero) must each fail a pin.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from workloads import Csx, csc_to_csr, csr_to_csc, er_csc, er_problem, identity, random_sparse


def _dense(x: Csx) -> tuple[np.ndarray, np.ndarray]:
    """Dense values and stored-pattern mask of a Csx."""
    d = np.zeros((x.nrows, x.ncols))
    mask = np.zeros((x.nrows, x.ncols), dtype=bool)
    for s in range(x.nmajor):
        for p in range(x.ptr[s], x.ptr[s + 1]):
            i, j = (x.idx[p], s) if x.fmt == "csc" else (s, x.idx[p])
            d[i, j] = x.val[p]
            mask[i, j] = True
    return d, mask


def _brute(a: Csx, b: Csx):
    """Pure-Python C = A*B: for each (i, j), products in ascending k, each
    added to the running sum as it comes.  Returns {(i, j): value}."""
    ad, am = _dense(a)
    bd, bm = _dense(b)
    out = {}
    for i in range(a.nrows):
        for j in range(b.ncols):
            s = None
            for k in range(a.ncols):
                if am[i, k] and bm[k, j]:
                    p = float(ad[i, k]) * float(bd[k, j])
                    s = p if s is None else s + p
            if s is not None:
                out[(i, j)] = s
    return out


def _as_dict(c: dict):
    out = {}
    rp, ci, cv = c["rowptr"], c["colidx"], c["val"]
    for i in range(len(rp) - 1):
        for p in range(rp[i], rp[i + 1]):
            out[(i, int(ci[p]))] = float(cv[p])
    return out


def _check_csr_canonical(c: dict):
    rp, ci = c["rowptr"], c["colidx"]
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == len(ci)
    for i in range(len(rp) - 1):
        seg = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(seg.astype(np.int64)) > 0)


def _matches_bruteforce(c: dict, a: Csx, b: Csx) -> bool:
    got = _as_dict(c)
    want = _brute(a, b)
    if set(got) != set(want):
        return False
    return all(got[key] == want[key] or (np.isnan(got[key]) and np.isnan(want[key])) for key in want)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _read_golden(name):
    """Parse a hand-worked fixture: dense A and B, then C's CSR and facts."""
    sections, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            head, *rest = line.split()
            if head in ("A", "B") and not rest:
                cur = sections.setdefault(head, [])
            elif head in ("rowptr", "colidx", "val", "absval", "flop"):
                sections[head] = [float(x) for x in rest]
                cur = None
            else:
                cur.append([float(x) for x in line.split()])
    return sections


@pytest.mark.parametrize("name", ["hand_worked_3x3.txt", "cancellation_1x2.txt"])
def test_hand_worked_golden(oracle_mod, name):
    g = _read_golden(name)
    a = _from_dense(np.array(g["A"]), "csc")
    b = _from_dense(np.array(g["B"]), "csr")
    c = oracle_mod.spgemm(a, b)
    _check_csr_canonical(c)
    assert list(c["rowptr"]) == [int(x) for x in g["rowptr"]]
    assert list(c["colidx"]) == [int(x) for x in g["colidx"]]
    assert list(c["val"]) == g["val"]
    if "absval" in g:
        assert list(c["absval"]) == g["absval"]
    assert c["flop"] == int(g["flop"][0])


def _from_dense(d: np.ndarray, fmt: str, keep_zero_mask=None) -> Csx:
    mask = d != 0 if keep_zero_mask is None else keep_zero_mask
    m, n = d.shape
    if fmt == "csc":
        ptr = [0]
        idx, val = [], []
        for j in range(n):
            for i in range(m):
                if mask[i, j]:
                    idx.append(i)
                    val.append(d[i, j])
            ptr.append(len(idx))
    else:
        ptr = [0]
        idx, val = [], []
        for i in range(m):
            for j in range(n):
                if mask[i, j]:
                    idx.append(j)
                    val.append(d[i, j])
            ptr.append(len(idx))
    return Csx(m, n, np.array(ptr, np.int64), np.array(idx, np.int32), np.array(val, np.float64), fmt)


CASES = [
    # (m, k, n, density, seed, values, extras)
    (17, 13, 11, 0.2, 1, "signed", {}),
    (30, 30, 30, 0.1, 2, "uniform", {}),
    (40, 25, 33, 0.15, 3, "signed", dict(a_dense_rows=(3,), b_dense_cols=(5,), a_empty_cols=(0, 7), b_empty_rows=(2,))),
    (1, 20, 1, 0.5, 4, "signed", {}),
    (25, 1, 25, 0.6, 5, "uniform", {}),
    (12, 9, 20, 0.0, 6, "uniform", {}),
    (20, 20, 20, 0.3, 7, "int", {}),
]


def _case(m, k, n, density, seed, values, extras):
    a = random_sparse(m, k, density, seed, "csc", values=values,
                      dense_rows=extras.get("a_dense_rows", ()), empty_cols=extras.get("a_empty_cols", ()))
    b = random_sparse(k, n, density, seed + 100, "csr", values=values,
                      dense_cols=extras.get("b_dense_cols", ()), empty_rows=extras.get("b_empty_rows", ()))
    return a, b


@pytest.mark.parametrize("case", CASES)
def test_bruteforce_tiny(oracle_mod, case):
    a, b = _case(*case)
    c = oracle_mod.spgemm(a, b)
    _check_csr_canonical(c)
    assert _matches_bruteforce(c, a, b)


def test_stored_zeros_and_cancellation(oracle_mod):
    # explicit stored zeros in the inputs and exact cancellations in C
    rng = np.random.default_rng(11)
    da = rng.integers(-2, 3, size=(15, 10)).astype(float)
    db = rng.integers(-2, 3, size=(10, 12)).astype(float)
    ma = rng.random((15, 10)) < 0.5
    mb = rng.random((10, 12)) < 0.5
    a = _from_dense(da * ma, "csc", keep_zero_mask=ma)  # some stored values are 0.0
    b = _from_dense(db * mb, "csr", keep_zero_mask=mb)
    c = oracle_mod.spgemm(a, b)
    assert _matches_bruteforce(c, a, b)
    # structure is the boolean product of the stored patterns
    pat = (ma.astype(int) @ mb.astype(int)) > 0
    got = np.zeros_like(pat)
    for (i, j) in _as_dict(c):
        got[i, j] = True
    assert np.array_equal(got, pat)
    assert np.any(pat & (da @ db == 0)), "the case should contain cancelled or zero-valued entries"


def test_integer_inputs_exact_vs_dense(oracle_mod):
    a = random_sparse(60, 50, 0.2, 21, "csc", values="int")
    b = random_sparse(50, 70, 0.2, 22, "csr", values="int")
    c = oracle_mod.spgemm(a, b)
    ad, am = _dense(a)
    bd, bm = _dense(b)
    want = ad @ bd  # exact: small integers
    pat = (am.astype(int) @ bm.astype(int)) > 0
    got = np.zeros_like(want)
    gmask = np.zeros_like(pat)
    for (i, j), v in _as_dict(c).items():
        got[i, j] = v
        gmask[i, j] = True
    assert np.array_equal(gmask, pat)
    assert np.array_equal(got, want)


def test_identity_right_and_left(oracle_mod):
    a = random_sparse(40, 30, 0.2, 31, "csc", values="signed")
    c = oracle_mod.spgemm(a, identity(30, "csr"))
    ar = csc_to_csr(a)
    assert np.array_equal(c["rowptr"], ar.ptr) and np.array_equal(c["colidx"], ar.idx)
    assert np.array_equal(c["val"], ar.val)
    assert len(c["colidx"]) == c["flop"]  # cf = 1 exactly
    b = random_sparse(30, 45, 0.2, 32, "csr", values="signed")
    c2 = oracle_mod.spgemm(identity(30, "csc"), b)
    assert np.array_equal(c2["rowptr"], b.ptr) and np.array_equal(c2["colidx"], b.idx)
    assert np.array_equal(c2["val"], b.val)


def test_permutation_and_diagonal(oracle_mod):
    n = 50
    rng = np.random.default_rng(41)
    perm = rng.permutation(n)
    # P with P(i, perm[i]) = 1  ->  (P B)(i, :) = B(perm[i], :)
    pmat = Csx(n, n, np.arange(n + 1, dtype=np.int64), perm.astype(np.int32), np.ones(n), "csr")
    b = random_sparse(n, 35, 0.2, 42, "csr", values="signed")
    c = oracle_mod.spgemm(csr_to_csc(pmat), b)
    for i in range(n):
        s, e = b.ptr[perm[i]], b.ptr[perm[i] + 1]
        assert np.array_equal(c["colidx"][c["rowptr"][i]:c["rowptr"][i + 1]], b.idx[s:e])
        assert np.array_equal(c["val"][c["rowptr"][i]:c["rowptr"][i + 1]], b.val[s:e])
    # diagonal scaling: (A D)(i, j) = A(i, j) * d_j, one product per entry
    a = random_sparse(n, n, 0.2, 43, "csc", values="signed")
    dvals = rng.random(n) + 0.5
    dmat = Csx(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), dvals, "csr")
    c = oracle_mod.spgemm(a, dmat)
    ar = csc_to_csr(a)
    assert np.array_equal(c["colidx"], ar.idx)
    assert np.array_equal(c["val"], ar.val * dvals[ar.idx])


def test_transpose_identity(oracle_mod):
    a = random_sparse(35, 28, 0.15, 51, "csc", values="signed")
    b = random_sparse(28, 41, 0.15, 52, "csr", values="signed")
    c = oracle_mod.spgemm(a, b)
    # B^T in CSC is B's CSR arrays; A^T in CSR is A's CSC arrays.
    ct = oracle_mod.spgemm(b.transpose_view(), a.transpose_view())
    # ct is C^T in CSR, i.e. C in CSC; compare entry sets bit for bit.
    d1 = _as_dict(c)
    d2 = {(j, i): v for (i, j), v in _as_dict(ct).items()}
    assert d1 == d2


def test_rows_entry_point_matches_full(oracle_mod):
    a, b = er_problem(2000, 5, 61, 62, values="signed")
    c = oracle_mod.spgemm(a, b)
    rows = np.array([0, 5, 1999, 77, 77, 1024], np.int64)
    r = oracle_mod.spgemm_rows(a, b, rows)
    for s, i in enumerate(rows):
        lo, hi = c["rowptr"][i], c["rowptr"][i + 1]
        assert np.array_equal(r["idx"][r["ptr"][s]:r["ptr"][s + 1]], c["colidx"][lo:hi])
        assert np.array_equal(r["val"][r["ptr"][s]:r["ptr"][s + 1]], c["val"][lo:hi])
        assert np.array_equal(r["absval"][r["ptr"][s]:r["ptr"][s + 1]], c["absval"][lo:hi])
    # all rows at once (rows=None) is C in CSR, bit for bit
    r = oracle_mod.spgemm_rows(a, b, None)
    for key, full in (("ptr", "rowptr"), ("idx", "colidx"), ("val", "val"), ("absval", "absval")):
        assert np.array_equal(r[key], c[full])


@pytest.mark.parametrize("n,d", [(4096, 4), (1000, 16), (300, 1), (64, 64)])
def test_flop_closed_form_er(oracle_mod, n, d):
    # exactly d per column of A: flop = d * nnz(B) = d * d * n (Algorithm 3)
    a, b = er_problem(n, d, 71, 72)
    assert oracle_mod.flop(a.ptr, b.ptr) == d * d * n
    c = oracle_mod.spgemm(a, b)
    assert c["flop"] == d * d * n
    assert len(c["colidx"]) <= c["flop"]  # cf >= 1


def test_er_expected_nnz(oracle_mod):
    # Poisson estimate E[nnz(C)] ~ n^2 (1 - exp(-d^2 / n)) for independent ER
    n, d = 4096, 4
    a, b = er_problem(n, d, 1, None)
    c = oracle_mod.spgemm(a, b)
    est = n * n * (1.0 - np.exp(-d * d / n))
    assert abs(len(c["colidx"]) - est) < 0.01 * est


def test_scipy_positive_inputs(oracle_mod):
    a = random_sparse(300, 200, 0.03, 81, "csc", values="uniform", dense_rows=(4,))
    b = random_sparse(200, 250, 0.03, 82, "csr", values="uniform", dense_cols=(9,))
    c = oracle_mod.spgemm(a, b)
    sa = sp.csc_matrix((a.val, a.idx, a.ptr), shape=(a.nrows, a.ncols))
    sb = sp.csr_matrix((b.val, b.idx, b.ptr), shape=(b.nrows, b.ncols))
    sc = (sa @ sb).tocsr()
    sc.sort_indices()
    assert np.array_equal(sc.indptr.astype(np.int64), c["rowptr"])
    assert np.array_equal(sc.indices, c["colidx"])
    assert np.allclose(sc.data, c["val"], rtol=1e-13, atol=0)


def test_mutations_are_caught(oracle_mod):
    """Plant plausible mistakes in copies of the oracle output; each must
    fail the brute-force pin."""
    a = random_sparse(20, 15, 0.3, 91, "csc", values="signed")
    b = random_sparse(15, 18, 0.3, 92, "csr", values="signed")
    c = oracle_mod.spgemm(a, b)
    assert _matches_bruteforce(c, a, b)

    # dropped term: remove one A entry before multiplying
    a2 = Csx(a.nrows, a.ncols, a.ptr.copy(), a.idx.copy(), a.val.copy(), "csc")
    a2.val[3] = 0.0
    bad = oracle_mod.spgemm(a2, b)
    assert not _matches_bruteforce(bad, a, b)

    # wrong sign on one value
    bad = {kk: v.copy() if isinstance(v, np.ndarray) else v for kk, v in c.items()}
    bad["val"][len(bad["val"]) // 2] *= -1.0
    assert not _matches_bruteforce(bad, a, b)

    # transposed operand: A^T used where A belongs (square shapes)
    sq_a = random_sparse(12, 12, 0.3, 93, "csc", values="signed")
    sq_b = random_sparse(12, 12, 0.3, 94, "csr", values="signed")
    wrong = oracle_mod.spgemm(csr_to_csc(Csx(12, 12, sq_a.ptr, sq_a.idx, sq_a.val, "csr")), sq_b)
    assert not _matches_bruteforce(wrong, sq_a, sq_b)

    # a lost structural entry (e.g. a cancelled sum dropped)
    bad = {kk: v.copy() if isinstance(v, np.ndarray) else v for kk, v in c.items()}
    i = int(np.argmax(np.diff(bad["rowptr"]) > 0))
    lo = bad["rowptr"][i]
    bad["colidx"] = np.delete(bad["colidx"], lo)
    bad["val"] = np.delete(bad["val"], lo)
    bad["rowptr"] = bad["rowptr"].copy()
    bad["rowptr"][i + 1:] -= 1
    assert not _matches_bruteforce(bad, a, b)

    # summation in another order is caught at the bit level on a crafted case:
    # 1e16 + 1 - 1e16 in ascending k gives 0, reversed gives 1.
    ca = _from_dense(np.array([[1e16, 1.0, -1e16]]), "csc")
    cb = _from_dense(np.array([[1.0], [1.0], [1.0]]), "csr")
    r = oracle_mod.spgemm(ca, cb)
    assert r["val"][0] == (1e16 + 1.0) + -1e16
