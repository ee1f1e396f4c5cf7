"""The bin-cut rule of the symbolic step, restated on the host (CPU only).

The device computes it inside a scan over the rows; this file states the rule in
plain numpy and checks the two bounds the packed key relies on, on
adversarial row-flop profiles: every bin of normal rows holds fewer than T
tuples, and at most 2^rowbits - 1 rows, so that the row part of a key,
(row in bin) << colbits, never reaches 2^rowbits - 1 and no real key equals
the all-ones sentinel that marks padding slots (also at column
2^colbits - 1 when n is a power of two).
"""
import numpy as np
import pytest


def bin_starts(rowflop: np.ndarray, T: int, rowbits: int) -> np.ndarray:
    """Rows that start a bin: the first row, a big row (flop > T/2) or the
    row after one, and every row whose weight g(r) = R[r] + c*r crosses a
    multiple of H = T - maxnormal, where maxnormal is the largest row flop
    <= T/2, cap = 2^rowbits - 1 and c = ceil(H / cap)."""
    m = rowflop.size
    R = np.concatenate([[0], np.cumsum(rowflop, dtype=np.int64)])
    thalf = T // 2
    normal = rowflop[rowflop <= thalf]
    maxnormal = int(normal.max()) if normal.size else 0
    H = T - maxnormal
    cap = (1 << rowbits) - 1
    c = max(1, -(-H // cap))
    r = np.arange(m, dtype=np.int64)
    g = R[:-1] + c * r
    start = np.zeros(m, bool)
    start[0] = True
    big = rowflop > thalf
    start[1:] |= big[1:] | big[:-1]
    start[1:] |= (g[1:] // H) != (g[:-1] // H)
    return np.flatnonzero(start)


def check_bins(rowflop, T, rowbits):
    starts = bin_starts(np.asarray(rowflop, np.int64), T, rowbits)
    ends = np.concatenate([starts[1:], [len(rowflop)]])
    R = np.concatenate([[0], np.cumsum(rowflop, dtype=np.int64)])
    for s, e in zip(starts, ends):
        tuples = R[e] - R[s]
        if e - s == 1 and rowflop[s] > T // 2:
            continue  # a big row is a bin by itself
        assert tuples < T, f"bin [{s},{e}) holds {tuples} tuples, tile {T}"
        assert e - s <= (1 << rowbits) - 1, f"bin [{s},{e}) holds {e - s} rows, rowbits {rowbits}"
    return starts


def test_empty_run_after_one_full_row():
    """The shape that once gave a bin of exactly 2^rowbits rows: T = 2048,
    n = 2^24 (rowbits 8), row 0 with 256 tuples (H = 1792) and 474 empty
    rows after it.  Row 475 would have been row 255 of bin [220, 476), and
    its key at column n-1 would have been 0xffffffff."""
    rf = np.zeros(576, np.int64)
    rf[0] = 256
    rf[475] = 1
    starts = check_bins(rf, 2048, 8)
    b = np.searchsorted(starts, 475, side="right") - 1
    rl = 475 - starts[b]
    assert (rl << 24) | ((1 << 24) - 1) != 0xFFFFFFFF


@pytest.mark.parametrize("rowbits", [1, 2, 5, 8, 11, 12])
@pytest.mark.parametrize("T", [256, 1000, 2048, 4096])
def test_random_profiles(rowbits, T):
    rng = np.random.default_rng(rowbits * 7919 + T)
    for trial in range(20):
        m = int(rng.integers(1, 5000))
        kind = trial % 4
        if kind == 0:  # mostly empty rows with sparse spikes
            rf = np.where(rng.random(m) < 0.02, rng.integers(1, T // 2 + 1, m), 0)
        elif kind == 1:  # uniform small rows
            rf = rng.integers(0, 8, m)
        elif kind == 2:  # some big rows
            rf = np.where(rng.random(m) < 0.05, rng.integers(T // 2 + 1, 3 * T, m), rng.integers(0, 40, m))
        else:  # all empty but one
            rf = np.zeros(m, np.int64)
            rf[int(rng.integers(0, m))] = int(rng.integers(1, T // 2 + 1))
        check_bins(rf, T, rowbits)


def test_all_empty_rows():
    check_bins(np.zeros(100000, np.int64), 2048, 4)
