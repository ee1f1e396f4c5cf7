// Row-range rounds and rows wider than one LDS tile.
//
// Rounds (the partitioned form of the method, Section 3.4 and the
// discussion of memory limits): when all tuples do not fit the workspace,
// the output rows are cut into ranges of consecutive bins and each range is
// expanded, sorted and compressed on its own.  A round with rows [r0, r1)
// uses, in every column of A, only the entries whose row lies in the range;
// rows are sorted inside each column, so that part is one contiguous
// sub-range found by binary search.
//
// Wide rows ("hub" rows, whose tuples exceed the tile T): after the expand,
// a wide row's tuples sit contiguously (a wide row is a bin by itself) in
// arbitrary column order.  They are partitioned by column window
// (2^wbits consecutive columns) into a second buffer.  Each (row, window)
// pair is a virtual row; virtual rows are cut into bins exactly like rows
// (a bin never spans two wide rows), with their own tile (at most 2048
// tuples), and sorted and compressed by the same kernels, with key =
// (virtual row in bin) << wbits | column in window.  A virtual row that
// alone exceeds that tile is summed in LDS by a dense accumulator over its
// 2^wbits columns instead of being sorted.
#pragma once
#include "pb_kernels.h"

namespace pb {

constexpr int kBigChunk = 65536;  // tuples of a wide row per partition workgroup
constexpr int kBigSub = 8192;     // tuples staged in LDS per partition step (one 512-thread workgroup per CU)
constexpr int kMaxLogWin = 10;    // at most 1024 windows per wide row
constexpr int kDenseBits = 12;    // dense accumulator: 4096 columns

// ---- rounds ---------------------------------------------------------------
__device__ __forceinline__ int64_t lower_bound_i32(const int32_t *a, int64_t lo, int64_t hi, int32_t x) {
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// astart[k] = first entry of A(:,k) with row >= r0; colflop[k] = entries of
// A(:,k) with row in [r0, r1) times the slots of a run of B(k,:).
__global__ __launch_bounds__(256) void k_round_cols(int64_t K, const int64_t *acp, const int32_t *ari,
                                                    const int64_t *brp, int32_t r0, int32_t r1, int align,
                                                    int64_t *astart, uint64_t *colflop) {
    const int64_t k = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (k >= K) return;
    const int64_t a0 = acp[k], a1 = acp[k + 1];
    const int64_t nb = brp[k + 1] - brp[k];
    int64_t s = a0, e = a0;
    if (nb > 0 && a1 > a0) {
        s = lower_bound_i32(ari, a0, a1, r0);
        e = lower_bound_i32(ari, s, a1, r1);
    }
    astart[k] = s;
    colflop[k] = (uint64_t)(e - s) * (uint64_t)run_slots(nb, align);
}

struct U64Src {
    const uint64_t *v;
    __device__ uint64_t operator()(int64_t i) const { return v[i]; }
};
struct U32Src {
    const uint32_t *v;
    __device__ uint64_t operator()(int64_t i) const { return v[i]; }
};

// ---- wide rows: partition by column window --------------------------------
struct BigArgs {
    int64_t nbig;             // wide rows in the round
    int lognwin, wbits, cb;   // windows per wide row = 2^lognwin, window = 2^wbits columns
    const int64_t *bigs;      // first tuple of wide row i (round-relative slot)
    const int64_t *bige;      // one past its last tuple
    const int64_t *cpre;      // partition chunks before wide row i (nbig + 1 entries)
    const uint32_t *keys;     // the round's tuples (wide rows: key = column; see TupleArr)
    const void *vals;
    int kstride;              // 32-bit words from one key to the next (TupleArr<VT>::kKeyStride)
    uint32_t *chist;          // per chunk: tuples per window (2^lognwin entries)
    uint32_t *cnt_v;          // per virtual row: tuples (zeroed before the histogram)
    uint32_t *cur_v;          // per virtual row: fill cursor (zeroed)
    const uint64_t *Rv;       // per virtual row: first slot in keys2 / vals2
    const RowTab *vrowtab;    // per virtual row: index inside its virtual bin
    uint32_t *keys2;
    void *vals2;
    int64_t nbigflop;         // size of keys2 / vals2
    uint32_t *err;
};

__device__ __forceinline__ void big_chunk_range(const BigArgs &a, int64_t c, int64_t &i, int64_t &s, int64_t &e) {
    i = last_le(a.cpre, 0, a.nbig, c);
    s = a.bigs[i] + (c - a.cpre[i]) * (int64_t)kBigChunk;
    const int64_t end = a.bige[i];
    e = s + kBigChunk < end ? s + kBigChunk : end;
}

// A wave's lanes hold consecutive tuples of a wide row, and a run's columns
// ascend, so neighbouring lanes often fall in the same window.  Lanes are
// grouped into segments of neighbours with the same window (lanes with no
// tuple carry kNoWin and form segments of their own); the head (first lane)
// of each segment does one LDS update for the whole segment.
constexpr uint32_t kNoWin = 0xffffffffu;
struct WinSegment {
    uint32_t head;  // first lane of this lane's segment
    uint32_t len;   // lanes in the segment (meaningful at the head)
    bool is_head;
};
__device__ __forceinline__ WinSegment win_segment(uint32_t win) {
    const uint32_t lane = lane_id();
    const uint32_t prev = __shfl_up(win, 1u, kWave);
    const uint64_t heads = ballot(lane == 0 || prev != win);
    const uint64_t upto = heads & ((2ull << lane) - 1ull);  // heads at or below this lane (lane 63: all)
    const uint64_t above = heads & ~((2ull << lane) - 1ull);
    WinSegment g;
    g.head = 63u - (uint32_t)__builtin_clzll(upto);
    g.is_head = g.head == lane;
    g.len = (above ? (uint32_t)__builtin_ctzll(above) : (uint32_t)kWave) - lane;
    return g;
}

// Tuples per window, per chunk (kept for the scatter) and per virtual row.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_big_hist(BigArgs a) {
    __shared__ uint32_t h[1 << kMaxLogWin];
    const int nwin = 1 << a.lognwin;
    int64_t i, s, e;
    big_chunk_range(a, blockIdx.x, i, s, e);
    for (int x = threadIdx.x; x < nwin; x += BLOCK) h[x] = 0;
    __syncthreads();
    const uint32_t colmask = a.cb ? ((1u << a.cb) - 1u) : 0u;
    // eight loads in flight per thread before their histogram updates
    constexpr int V = 8;
    for (int64_t p0 = s; p0 < e; p0 += (int64_t)V * BLOCK) {
        uint32_t kk[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int64_t p = p0 + v * BLOCK + threadIdx.x;
            kk[v] = p < e ? a.keys[p * a.kstride] : kSentinel;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const uint32_t win = kk[v] != kSentinel ? (kk[v] & colmask) >> a.wbits : kNoWin;
            const WinSegment g = win_segment(win);
            if (g.is_head && win != kNoWin) atomicAdd(&h[win], g.len);
        }
    }
    __syncthreads();
    uint32_t *ch = a.chist + (int64_t)blockIdx.x * nwin;
    for (int x = threadIdx.x; x < nwin; x += BLOCK) {
        const uint32_t c = h[x];
        ch[x] = c;
        if (c) atomic_add_agent(&a.cnt_v[(i << a.lognwin) + x], c);
    }
}

// Scatter one chunk into its virtual rows.  The chunk reserves, per window,
// a contiguous range of the virtual row with one atomic; inside the chunk,
// steps of kBigSub tuples are ordered by window in LDS and written as runs.
template <int BLOCK, class VT>
__global__ __launch_bounds__(BLOCK) void k_big_scatter(BigArgs a) {
    constexpr int NWMAX = 1 << kMaxLogWin;
    constexpr int PER = kBigSub / BLOCK;
    constexpr int WPT = NWMAX / BLOCK;
    static_assert(kBigSub % BLOCK == 0 && NWMAX % BLOCK == 0, "shape");
    __shared__ uint32_t cbase[NWMAX];  // per window: first slot, relative to the row's first virtual row
    __shared__ uint32_t rlw[NWMAX];
    __shared__ uint32_t run[NWMAX];
    __shared__ uint32_t hsc[NWMAX];
    __shared__ uint32_t hoff[NWMAX];
    __shared__ uint32_t skey[kBigSub];
    __shared__ uint16_t swin[kBigSub];
    __shared__ VT sval[kBigSub];
    __shared__ uint64_t s_scan[BLOCK / kWave + 1];
    const int nwin = 1 << a.lognwin;
    int64_t i, s, e;
    big_chunk_range(a, blockIdx.x, i, s, e);
    const int64_t vbase = (int64_t)a.Rv[i << a.lognwin];  // the row's tuples: fewer than 2^32 after it
    const uint32_t *ch = a.chist + (int64_t)blockIdx.x * nwin;
    for (int x = threadIdx.x; x < nwin; x += BLOCK) {
        const uint32_t c = ch[x];
        run[x] = 0;
        if (c) {
            const int64_t v = (i << a.lognwin) + x;
            const uint32_t off = atomic_add_agent(&a.cur_v[v], c);
            cbase[x] = (uint32_t)((int64_t)a.Rv[v] - vbase) + off;
            rlw[x] = a.vrowtab[v].rl << a.wbits;
        }
    }
    const uint32_t colmask = a.cb ? ((1u << a.cb) - 1u) : 0u;
    const uint32_t wmask = (1u << a.wbits) - 1u;
    const TupleArr<VT> in((void *)a.keys, (void *)a.vals);
    const TupleArr<VT> out((void *)a.keys2, a.vals2);
    for (int64_t s0 = s; s0 < e; s0 += kBigSub) {
        const int nsub = (int)((e - s0) < kBigSub ? (e - s0) : kBigSub);
        for (int x = threadIdx.x; x < nwin; x += BLOCK) hsc[x] = 0;
        __syncthreads();
        uint32_t col[PER], rank[PER];
        bool real[PER];
        VT val[PER];
        // unconditional loads (the last tuple stands in past the end) overlap
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = u * BLOCK + threadIdx.x;
            col[u] = in.key(s0 + (q < nsub ? q : nsub - 1));
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = u * BLOCK + threadIdx.x;
            val[u] = in.val(s0 + (q < nsub ? q : nsub - 1));
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int q = u * BLOCK + threadIdx.x;
            real[u] = q < nsub && col[u] != kSentinel;  // padding slots are dropped here
            col[u] &= colmask;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const uint32_t win = real[u] ? col[u] >> a.wbits : kNoWin;
            const WinSegment g = win_segment(win);
            uint32_t base = 0;
            if (g.is_head && win != kNoWin) base = atomicAdd(&hsc[win], g.len);
            rank[u] = (uint32_t)__shfl((int)base, (int)g.head, kWave) + (lane_id() - g.head);
        }
        __syncthreads();
        // exclusive scan of the step's window counts
        uint32_t cnt[WPT];
        uint64_t tsum = 0;
#pragma unroll
        for (int x = 0; x < WPT; ++x) {
            const int wdx = threadIdx.x * WPT + x;
            cnt[x] = wdx < nwin ? hsc[wdx] : 0u;
            tsum += cnt[x];
        }
        uint64_t total;
        uint64_t ex = block_excl_scan<BLOCK, SumOp>(tsum, s_scan, total);
        const int nput = (int)total;  // real tuples of the step
#pragma unroll
        for (int x = 0; x < WPT; ++x) {
            const int wdx = threadIdx.x * WPT + x;
            if (wdx < nwin) hoff[wdx] = (uint32_t)ex;
            ex += cnt[x];
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            if (real[u]) {
                const uint32_t w = col[u] >> a.wbits;
                const uint32_t pos = hoff[w] + rank[u];
                skey[pos] = rlw[w] | (col[u] & wmask);
                swin[pos] = (uint16_t)w;
                sval[pos] = val[u];
            }
        }
        __syncthreads();
        for (int q = threadIdx.x; q < nput; q += BLOCK) {
            const uint32_t w = swin[q];
            const int64_t dest = vbase + (int64_t)cbase[w] + run[w] + (q - (int)hoff[w]);
            if ((uint64_t)dest < (uint64_t)a.nbigflop) {
                out.put(dest, skey[q], sval[q]);
            } else {
                atomic_or_agent(a.err, (uint32_t)kErrBinOverflow);
            }
        }
        __syncthreads();
        for (int x = threadIdx.x; x < nwin; x += BLOCK) run[x] += hsc[x];
        __syncthreads();
    }
}

// ---- wide rows: virtual-row sums and pointers ------------------------------
// nnz of wide row i = sum of its virtual rows' counts.  One wave per row.
__global__ __launch_bounds__(256) void k_big_rowsum(int64_t nbig, int lognwin, const int32_t *bigr, int64_t row_base,
                                                    const uint32_t *rownnz_v, uint32_t *rownnz) {
    const int64_t i = blockIdx.x * (int64_t)4 + threadIdx.x / kWave;
    if (i >= nbig) return;
    const uint32_t lane = lane_id();
    const int nwin = 1 << lognwin;
    uint64_t sum = 0;
    for (int w = (int)lane; w < nwin; w += kWave) sum += rownnz_v[(i << lognwin) + w];
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) sum += __shfl_xor(sum, d, kWave);
    if (lane == 0) rownnz[bigr[i] - row_base] = (uint32_t)sum;
}

// rowptr_v[(i, w)] = C's row pointer of wide row i + entries of its earlier
// windows.  One wave per row.
__global__ __launch_bounds__(256) void k_big_rowptr(int64_t nbig, int lognwin, const int32_t *bigr, int64_t row_base,
                                                    const int64_t *rowptr, const uint32_t *rownnz_v,
                                                    int64_t *rowptr_v) {
    const int64_t i = blockIdx.x * (int64_t)4 + threadIdx.x / kWave;
    if (i >= nbig) return;
    const uint32_t lane = lane_id();
    const int nwin = 1 << lognwin;
    int64_t run = rowptr[bigr[i] - row_base];
    for (int w0 = 0; w0 < nwin; w0 += kWave) {
        const int w = w0 + (int)lane;
        const uint64_t c = w < nwin ? rownnz_v[(i << lognwin) + w] : 0u;
        const uint64_t inc = wave_incl_scan<SumOp>(c);
        if (w < nwin) rowptr_v[(i << lognwin) + w] = run + (int64_t)(inc - c);
        run += (int64_t)__shfl(inc, kWave - 1, kWave);
    }
}

// ---- wide rows: dense accumulation of one window ---------------------------
// For a virtual row with more tuples than the virtual tile: a bitmap of the
// window's columns marks every position hit (so cancelled sums stay stored), and
// (OUT) a double accumulator per column receives every tuple by an LDS
// atomic add.  Count mode writes the number of marked columns; output mode
// writes the marked columns in order at the virtual row's place in C.
// Workgroups take the listed virtual rows in turn.
struct DenseArgs {
    const int32_t *list;      // virtual rows to do
    const uint64_t *count;    // how many
    const uint64_t *Rv;
    const uint32_t *keys2;  // see TupleArr
    const void *vals2;
    int wbits, lognwin;
    uint32_t *rownnz_v;       // count mode
    const int64_t *rowptr_v;  // output mode
    int32_t *colidx;
    void *cvals;
    int64_t capacity;
    uint32_t *err;
};

template <int BLOCK, class VT, bool OUT>
__global__ __launch_bounds__(BLOCK) void k_dense(DenseArgs a) {
    constexpr int WD = 1 << kDenseBits;
    constexpr int CPT = WD / BLOCK;  // columns per thread
    static_assert(CPT == 8, "two flag words per thread");
    __shared__ double acc[OUT ? WD : 1];
    __shared__ uint32_t hitw[WD / 4];  // one flag byte per column: 1 when some tuple hits it
    uint8_t *hit = (uint8_t *)hitw;
    __shared__ uint64_t s_scan[BLOCK / kWave + 1];
    if (a.wbits > kDenseBits) {
        if (threadIdx.x == 0 && *a.count > 0) atomic_or_agent(a.err, (uint32_t)kErrWide);
        return;
    }
    const int64_t cnt = (int64_t)*a.count;
    const uint32_t wmask = (1u << a.wbits) - 1u;
    const int ncol = 1 << a.wbits;
    const TupleArr<VT> tv((void *)a.keys2, (void *)a.vals2);
    VT *cv = (VT *)a.cvals;
    for (int64_t it = blockIdx.x; it < cnt; it += gridDim.x) {
        const int64_t v = a.list[it];
        const int64_t s = (int64_t)a.Rv[v], e = (int64_t)a.Rv[v + 1];
        for (int x = threadIdx.x; x < WD / 4; x += BLOCK) hitw[x] = 0;
        if (OUT)
            for (int x = threadIdx.x; x < ncol; x += BLOCK) acc[x] = 0.0;
        __syncthreads();
        constexpr int U = 8;  // tuples loaded per thread before they are added
        for (int64_t p0 = s + threadIdx.x; p0 < e; p0 += (int64_t)BLOCK * U) {
            uint32_t kc[U];
            VT vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = p0 + u * BLOCK < e ? p0 + u * BLOCK : e - 1;
                kc[u] = tv.key(q);
                if (OUT) vv[u] = tv.val(q);
            }
            // lanes past the end repeat the last tuple with nothing to add
            // (its column is hit anyway), so every use of the loads is
            // unconditional and they stay overlapped; the flags are plain
            // byte stores (every writer stores 1)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in = p0 + u * BLOCK < e;
                const uint32_t c = kc[u] & wmask;
                hit[c] = 1;
                if (OUT) atomicAdd(&acc[c], in ? (double)vv[u] : 0.0);
            }
        }
        __syncthreads();
        // this thread's 8 columns as a bit mask
        const uint64_t f8 = ((uint64_t)hitw[2 * threadIdx.x + 1] << 32) | hitw[2 * threadIdx.x];
        uint32_t byte = 0;
#pragma unroll
        for (int x = 0; x < CPT; ++x) byte |= (uint32_t)((f8 >> (8 * x)) & 1u) << x;
        const uint32_t mine = (uint32_t)__builtin_popcount(byte);
        uint64_t total;
        const uint64_t ex = block_excl_scan<BLOCK, SumOp>(mine, s_scan, total);
        if (!OUT) {
            if (threadIdx.x == 0) a.rownnz_v[v] = (uint32_t)total;
        } else {
            int64_t out = a.rowptr_v[v] + (int64_t)ex;
            const uint32_t colbase = ((uint32_t)(v & ((1 << a.lognwin) - 1))) << a.wbits;
            for (int x = 0; x < CPT; ++x) {
                if (byte & (1u << x)) {
                    const uint32_t c = threadIdx.x * CPT + x;
                    if (out < a.capacity) {
                        a.colidx[out] = (int32_t)(colbase | c);
                        cv[out] = (VT)acc[c];
                    } else {
                        atomic_or_agent(a.err, (uint32_t)kErrCapacity);
                    }
                    ++out;
                }
            }
        }
        __syncthreads();
    }
}

}  // namespace pb
