// PB-SpGEMM kernels for gfx950 (wave64).  No MFMA: nothing here is a dense
// contraction.  Every phase streams HBM; the per-bin sort runs in LDS.
#pragma once
#include "pb_device.h"

namespace pb {

// ---------------------------------------------------------------------------
// Facts the symbolic step leaves on the device (read back once).
// Per-row facts: R[r], the first slot of the row's share of the tuple
// array (bins are consecutive slot ranges in row order; inside a bin the
// runs of its rows may be interleaved), and the row's index inside its bin.
struct RowTab {
    int64_t base;
    uint32_t rl;
    uint32_t bin;
};

struct SymInfo {
    uint64_t flop;       // Algorithm 3's multiplication count
    uint64_t slots;      // tuple slots: runs rounded up to the run alignment
    uint64_t nbins;      // bins of consecutive rows
    uint64_t maxnormal;  // largest row flop among rows <= tile/2
    uint64_t maxrow;     // largest row flop
    uint64_t noversize;  // rows with more tuples than the tile
    uint64_t maxbin;     // tuple slots of the largest bin
    uint32_t err;
    uint32_t pad;
};

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// Scan in two launches (reduce, then scan): k_scan_tiles writes each tile's
// total, k_scan_apply combines the totals of the tiles before its own (in
// tile order) and scans its tile.  With many tiles, that combination would
// grow with the square of the tile count, so k_scan_parts (one workgroup)
// first turns the totals into exclusive prefixes in place and each tile
// reads its own.  No tile waits for another, so nothing
// depends on the order in which workgroups start; a single-pass scan would
// need every tile to take a ticket from one device-wide counter, and on
// this chip's eight XCDs those tickets serialise.  Thread t of a tile owns
// IPT consecutive elements.  Src(i) -> element payload; Dst(i, exclusive,
// element) stores results; Dst::total(t) receives the grand total (called by
// the owner of the last element); Dst::side(i, e) -> value max-reduced per
// tile and handed to Dst::side_commit.  Op may be non-commutative: every
// combination is made in element order.
template <int BLOCK, int IPT, class Op, class Src>
__global__ __launch_bounds__(BLOCK) void k_scan_tiles(int64_t n, Src src, uint64_t *part) {
    constexpr int NW = BLOCK / kWave;
    __shared__ uint64_t s_tmp[NW + 1];
    const int64_t base = blockIdx.x * (int64_t)(BLOCK * IPT) + (int64_t)threadIdx.x * IPT;
    uint64_t e[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) e[j] = base + j < n ? src(base + j) : Op::identity();
    uint64_t local = Op::identity();
#pragma unroll
    for (int j = 0; j < IPT; ++j) local = Op::combine(local, e[j]);
    uint64_t tile_total;
    block_excl_scan<BLOCK, Op>(local, s_tmp, tile_total);
    if (threadIdx.x == 0) part[blockIdx.x] = tile_total;
}

// Exclusive scan of the tile totals in place, by one workgroup, in chunks
// of BLOCK * 8 carried in tile order.
template <int BLOCK, class Op>
__global__ __launch_bounds__(BLOCK) void k_scan_parts(int64_t tiles, uint64_t *part) {
    constexpr int NW = BLOCK / kWave;
    constexpr int PPT = 8;
    __shared__ uint64_t s_tmp[NW + 1];
    uint64_t carry = Op::identity();
    for (int64_t c0 = 0; c0 < tiles; c0 += (int64_t)BLOCK * PPT) {
        const int64_t base = c0 + (int64_t)threadIdx.x * PPT;
        uint64_t e[PPT];
        uint64_t local = Op::identity();
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            e[j] = base + j < tiles ? part[base + j] : Op::identity();
            local = Op::combine(local, e[j]);
        }
        uint64_t tot;
        uint64_t run = Op::combine(carry, block_excl_scan<BLOCK, Op>(local, s_tmp, tot));  // has barriers
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            if (base + j < tiles) part[base + j] = run;
            run = Op::combine(run, e[j]);
        }
        carry = Op::combine(carry, tot);
    }
}

// prefixed: part[t] already holds the combination of the tiles before t.
template <int BLOCK, int IPT, class Op, class Src, class Dst>
__global__ __launch_bounds__(BLOCK) void k_scan_apply(int64_t n, Src src, Dst dst, const uint64_t *part,
                                                      int prefixed) {
    constexpr int NW = BLOCK / kWave;
    __shared__ uint64_t s_tmp[NW + 1];
    __shared__ uint64_t s_side[NW];
    const int64_t tile = blockIdx.x;
    const int64_t base = tile * (int64_t)(BLOCK * IPT) + (int64_t)threadIdx.x * IPT;
    uint64_t e[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) e[j] = base + j < n ? src(base + j) : Op::identity();
    // the tiles before this one: their prefix, or (few tiles) thread t
    // combines a consecutive range of their totals and the block combines
    // the threads in order
    uint64_t before;
    if (prefixed) {
        before = part[tile];
    } else {
        const int64_t per = (tile + BLOCK - 1) / BLOCK;
        const int64_t t0 = (int64_t)threadIdx.x * per;
        const int64_t t1 = t0 + per < tile ? t0 + per : tile;
        uint64_t pre = Op::identity();
        for (int64_t x = t0; x < t1; ++x) pre = Op::combine(pre, part[x]);
        block_excl_scan<BLOCK, Op>(pre, s_tmp, before);
    }
    uint64_t local = Op::identity();
    uint64_t side = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t i = base + j;
        if (i < n) {
            const uint64_t sv = dst.side(i, e[j]);
            side = sv > side ? sv : side;
        }
        local = Op::combine(local, e[j]);
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const uint64_t o = __shfl_xor(side, d, kWave);
        side = o > side ? o : side;
    }
    if (lane_id() == 0) s_side[threadIdx.x / kWave] = side;
    uint64_t tile_total;
    const uint64_t texcl = block_excl_scan<BLOCK, Op>(local, s_tmp, tile_total);  // has barriers
    if (threadIdx.x == 0) {
        uint64_t mx = 0;
        for (int w = 0; w < NW; ++w) mx = s_side[w] > mx ? s_side[w] : mx;
        dst.side_commit(mx);
    }
    uint64_t run = Op::combine(before, texcl);
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t i = base + j;
        if (i < n) dst(i, run, e[j]);
        run = Op::combine(run, e[j]);
    }
    if (base < n && base + IPT >= n) dst.total(run);
}

struct NoSide {
    __device__ uint64_t side(int64_t, uint64_t) const { return 0; }
    __device__ void side_commit(uint64_t) const {}
};

// Where each A entry's run goes, one 64-bit word per entry: the run's first
// tuple slot in the low 40 bits, the run's row inside its bin above them.
// Bins therefore hold fewer than 2^24 rows, and products fewer than 2^40
// tuple slots.
constexpr int kEntSlotBits = 40;
constexpr uint64_t kEntSlotMask = (1ull << kEntSlotBits) - 1;
constexpr int kMaxBinRowBits = 64 - kEntSlotBits;
__device__ __forceinline__ uint64_t ent_pack(uint64_t slot, uint32_t rl) {
    return slot | ((uint64_t)rl << kEntSlotBits);
}

// Runs (the tuples of one A entry) occupy a multiple of `align` slots, so
// that runs written by different waves never share a 32-byte sector of the
// tuple arrays; the slots past a run's end hold the sentinel key.
__device__ __forceinline__ int64_t run_slots(int64_t nb, int align) {
    return (nb + align - 1) / align * align;
}

// Tuple arrays.  FP64 tuples are two arrays (32-bit keys, double values).
// FP32c tuples are one array of 8-byte words, key in the low half and the
// float value's bits in the high half, so the run of tuples an A entry
// writes is one contiguous segment.  Built from the (keys, vals) pair of a
// workspace layout; for FP32c `keys` points at the word array and `vals` is
// unused.
template <class VT>
struct TupleArr;
template <>
struct TupleArr<double> {
    uint32_t *k;
    double *v;
    static constexpr int kKeyStride = 1;  // 32-bit words from one key to the next
    __device__ TupleArr(void *keys, void *vals) : k((uint32_t *)keys), v((double *)vals) {}
    __device__ void put(int64_t i, uint32_t key, double val) const {
        k[i] = key;
        v[i] = val;
    }
    __device__ uint32_t key(int64_t i) const { return k[i]; }
    __device__ double val(int64_t i) const { return v[i]; }
};
template <>
struct TupleArr<float> {
    uint2 *t;
    static constexpr int kKeyStride = 2;
    __device__ TupleArr(void *keys, void *) : t((uint2 *)keys) {}
    __device__ void put(int64_t i, uint32_t key, float val) const { t[i] = make_uint2(key, __float_as_uint(val)); }
    __device__ uint32_t key(int64_t i) const { return t[i].x; }
    __device__ float val(int64_t i) const { return __uint_as_float(t[i].y); }
};

// Algorithm 3: flop_k = nnz(A(:,k)) * nnz(B(k,:)); F = exclusive scan of
// the column's tuple slots, nnz(A(:,k)) * run_slots(nnz(B(k,:))).
struct ColFlopSrc {
    const int64_t *acp, *brp;
    int align;
    __device__ uint64_t operator()(int64_t k) const {
        return (uint64_t)((acp[k + 1] - acp[k]) * run_slots(brp[k + 1] - brp[k], align));
    }
};
struct ColFlopDst : NoSide {
    int64_t *F;
    int64_t K;
    SymInfo *info;
    __device__ void operator()(int64_t k, uint64_t excl, uint64_t) const { F[k] = (int64_t)excl; }
    __device__ void total(uint64_t t) const {
        F[K] = (int64_t)t;
        info->slots = t;
    }
};

// Per-row flop: rowflop[r] = sum over k with A(r,k) stored of nnz(B(k,:)).
// The counter update for A entry e returns the flop already counted in its
// row, which becomes the offset of e's run inside the row's tuple range
// (runpos[e]); the expand then writes every run to a fixed place without
// atomics.  One thread per column of A; columns longer than 32 entries are
// taken by the whole wave, lanes striding over the column.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_rowflop(int64_t K, const int64_t *acp, const int32_t *ari,
                                                   const int64_t *brp, int align, uint64_t *rowflop,
                                                   uint32_t *runpos, SymInfo *info) {
    const int64_t k = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    int64_t a0 = 0, na = 0, nb = 0, pnb = 0;
    if (k < K) {
        a0 = acp[k];
        na = acp[k + 1] - a0;
        nb = brp[k + 1] - brp[k];
        if (nb == 0) na = 0;
        pnb = run_slots(nb, align);
    }
    // Algorithm 3's multiplication count, one atomic per wave
    uint64_t f = (uint64_t)(na * nb);
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) f += __shfl_xor(f, d, kWave);
    if (lane_id() == 0 && f) atomic_add_agent(&info->flop, f);
    const bool longcol = na > 32;
    if (!longcol) {
        for (int64_t e = a0; e < a0 + na; ++e)
            runpos[e] = (uint32_t)atomic_add_agent(&rowflop[ari[e]], (uint64_t)pnb);
    }
    uint64_t mask = ballot(longcol);
    const uint32_t lane = lane_id();
    while (mask) {
        const int L = __builtin_ctzll(mask);
        mask &= mask - 1;
        const int64_t la0 = __shfl(a0, L, kWave);
        const int64_t lna = __shfl(na, L, kWave);
        const int64_t lnb = __shfl(pnb, L, kWave);
        for (int64_t e = la0 + lane; e < la0 + lna; e += kWave)
            runpos[e] = (uint32_t)atomic_add_agent(&rowflop[ari[e]], (uint64_t)lnb);
    }
}

// ---------------------------------------------------------------------------
// Per-row flop and run offsets without device atomics (products with fewer
// than 2^32 entries in A and at most 2^25 rows).  The rows are cut into
// buckets of kRowBucketRows consecutive rows.  A counting sort distributes
// the entries of A to their row's bucket: each workgroup of the distribution
// takes a contiguous range of entries (read in order, so every pass over
// them is coalesced), builds an LDS histogram of their buckets, a scan of
// the bucket-major histogram gives every (bucket, workgroup) pair its place,
// and a second pass writes one record per entry there (and the record's
// place, per entry).  One workgroup per bucket adds each record's run slots
// to its row's LDS counter (the per-row tuple counts).  After the row scan
// and the bin cut, one workgroup per bucket gives each record its run's
// place inside its bin (an LDS cursor per part of a bin), and a last pass
// over the entry ranges copies each entry's place: the records of one range
// sit in one short segment per bucket, so these reads, like every write,
// are whole lines.  The same bins as k_rowflop's; only the order of the
// runs inside a bin differs.
constexpr int kRowBucketBits = 12;
constexpr int kRowBucketRows = 1 << kRowBucketBits;
constexpr int kMaxRowBuckets = 8192;      // LDS histogram of the distribution
constexpr int kBucketBlock = 512;         // threads of the distribution passes
constexpr int kBucketCols = 4032;         // columns of a range held in LDS
constexpr uint32_t kRunField = 0xfffffu;  // 20-bit run-slot field; saturated:
                                          // recomputed from B's row pointers
struct RowBucketArgs {
    int64_t K, nnz;
    const int64_t *acp, *brp;
    const int32_t *ari;
    int align;
    int64_t epw;      // entries per workgroup of the distribution passes
    int nbkt, ngrp;   // buckets; workgroups of the distribution passes
    int64_t cpw;      // columns per workgroup for the flop and range starts
    int32_t *kstart;  // [ngrp + 1]: column holding entry g * epw; [ngrp]: the
                      // column holding the last entry
    uint32_t *hist;   // nbkt x ngrp counts (bucket-major), then their scan
    uint64_t *gflop;  // [ngrp]: multiplications of each workgroup's columns
    uint32_t *rec;    // bucket order: row in bucket | run slots << 12
    uint32_t *roff;   // bucket order: the column when the slots field is
                      // saturated, then the run's offset in its row
    uint32_t *posof;  // per entry: its record
    uint64_t *rowflop;
    SymInfo *info;
    const RowTab *rowtab;  // per row: first slot and row inside its bin
    uint64_t *entrec;             // bucket order: the record's run destination (ent_pack)
    uint64_t *ent;                // entry order: the entry's run destination
    // fixed order only (null otherwise)
    uint32_t *recent;             // bucket order: the record's entry of A
    uint32_t *lste, *lsts, *lstp; // per bucket, grouped by row: entry, run slots, record
    int64_t det_tmax;             // the tile: wider rows are not ordered
};

template <int BLOCK>
__device__ __forceinline__ uint64_t block_sum(uint64_t v, uint64_t *lds) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    if (lane_id() == 0) lds[threadIdx.x / kWave] = v;
    __syncthreads();
    uint64_t t = 0;
    for (int i = 0; i < BLOCK / kWave; ++i) t += lds[i];
    __syncthreads();
    return t;
}

// Pass 1 (dynamic LDS: one counter per bucket).  Also, over a slice of the
// columns: their multiplications (Algorithm 3) and each entry range's first
// column.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_bucket_hist(RowBucketArgs a) {
    extern __shared__ uint32_t s_h[];
    __shared__ uint64_t s_red[BLOCK / kWave];
    for (int b = threadIdx.x; b < a.nbkt; b += BLOCK) s_h[b] = 0;
    __syncthreads();
    const int64_t e0 = blockIdx.x * a.epw;
    const int64_t e1 = e0 + a.epw < a.nnz ? e0 + a.epw : a.nnz;
    constexpr int U = 4;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += (int64_t)BLOCK * U) {
        int32_t r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = a.ari[e + u * BLOCK < e1 ? e + u * BLOCK : e1 - 1];  // loads overlap
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e + u * BLOCK < e1) atomicAdd(&s_h[r[u] >> kRowBucketBits], 1u);
    }
    uint64_t f = 0;
    const int64_t c1 = (blockIdx.x + 1) * a.cpw < a.K ? (blockIdx.x + 1) * a.cpw : a.K;
    for (int64_t c = blockIdx.x * a.cpw + threadIdx.x; c < c1; c += BLOCK) {
        const int64_t a0 = a.acp[c], a1 = a.acp[c + 1];
        f += (uint64_t)((a1 - a0) * (a.brp[c + 1] - a.brp[c]));
        for (int64_t g = (a0 + a.epw - 1) / a.epw; g * a.epw < a1; ++g) a.kstart[g] = (int32_t)c;
        if (a0 <= a.nnz - 1 && a.nnz - 1 < a1) a.kstart[a.ngrp] = (int32_t)c;
    }
    f = block_sum<BLOCK>(f, s_red);
    if (threadIdx.x == 0) a.gflop[blockIdx.x] = f;
    for (int b = threadIdx.x; b < a.nbkt; b += BLOCK) a.hist[(int64_t)b * a.ngrp + blockIdx.x] = s_h[b];
}

// Pass 2: the same entry ranges; an entry's column comes from a binary
// search of the range's column starts in LDS (or, for a range spanning more
// than kBucketCols columns, from walking those columns).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_bucket_scatter(RowBucketArgs a) {
    extern __shared__ uint32_t s_cur[];
    __shared__ uint32_t s_off[kBucketCols + 1];
    __shared__ uint32_t s_slots[kBucketCols];
    for (int b = threadIdx.x; b < a.nbkt; b += BLOCK) s_cur[b] = a.hist[(int64_t)b * a.ngrp + blockIdx.x];
    const int64_t e0 = blockIdx.x * a.epw;
    const int64_t e1 = e0 + a.epw < a.nnz ? e0 + a.epw : a.nnz;
    const int64_t k0 = a.kstart[blockIdx.x], kend = a.kstart[blockIdx.x + 1];
    const int64_t nc = kend - k0 + 1;
    auto put = [&](int64_t e, int32_t r, uint32_t field, int64_t k) {
        const uint32_t pos = atomicAdd(&s_cur[r >> kRowBucketBits], 1u);
        a.rec[pos] = (uint32_t)(r & (kRowBucketRows - 1)) | field << kRowBucketBits;
        if (field == kRunField) a.roff[pos] = (uint32_t)k;
        a.posof[e] = pos;
        if (a.recent) a.recent[pos] = (uint32_t)e;
    };
    if (nc <= kBucketCols) {
        for (int64_t i = threadIdx.x; i <= nc; i += BLOCK) {
            const int64_t c = k0 + i;
            const int64_t o = a.acp[c] - e0;
            s_off[i] = (uint32_t)(o < 0 ? 0 : (o > a.epw ? a.epw : o));
            if (i < nc) {
                const int64_t sl = run_slots(a.brp[c + 1] - a.brp[c], a.align);
                s_slots[i] = sl < (int64_t)kRunField ? (uint32_t)sl : kRunField;
            }
        }
        __syncthreads();
        constexpr int U = 4;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += (int64_t)BLOCK * U) {
            int32_t r[U];
#pragma unroll
            for (int u = 0; u < U; ++u) r[u] = a.ari[e + u * BLOCK < e1 ? e + u * BLOCK : e1 - 1];  // loads overlap
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (e + u * BLOCK >= e1) continue;
                const uint32_t rel = (uint32_t)(e + u * BLOCK - e0);
                // s_off[lo] <= rel < s_off[hi]
                int lo = 0, hi = (int)nc;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_off[mid] <= rel) lo = mid;
                    else hi = mid;
                }
                put(e + u * BLOCK, r[u], s_slots[lo], k0 + lo);
            }
        }
    } else {
        __syncthreads();
        for (int64_t c = k0 + threadIdx.x; c <= kend; c += BLOCK) {
            const int64_t c0 = a.acp[c], c1 = a.acp[c + 1];
            const int64_t sl = run_slots(a.brp[c + 1] - a.brp[c], a.align);
            const uint32_t field = sl < (int64_t)kRunField ? (uint32_t)sl : kRunField;
            for (int64_t e = c0 > e0 ? c0 : e0; e < (c1 < e1 ? c1 : e1); ++e) put(e, a.ari[e], field, c);
        }
    }
}

// Pass 3: one workgroup per bucket sums its records' slots per row (the
// rows' tuple counts for the row scan and the bin cut); block 0 also adds up
// the multiplication count.  roff keeps the column of saturated records.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_bucket_count(RowBucketArgs a, int64_t m) {
    __shared__ unsigned long long s_cnt[kRowBucketRows];
    __shared__ uint64_t s_red[BLOCK / kWave];
    for (int i = threadIdx.x; i < kRowBucketRows; i += BLOCK) s_cnt[i] = 0;
    const int64_t b = blockIdx.x;
    if (b == 0) {
        uint64_t f = 0;
        for (int g = threadIdx.x; g < a.ngrp; g += BLOCK) f += a.gflop[g];
        f = block_sum<BLOCK>(f, s_red);
        if (threadIdx.x == 0) a.info->flop = f;
    }
    __syncthreads();
    const uint32_t p0 = a.hist[b * a.ngrp], p1 = a.hist[(b + 1) * a.ngrp];
    constexpr int U = 4;
    for (int64_t p = (int64_t)p0 + threadIdx.x; p < p1; p += (int64_t)BLOCK * U) {
        uint32_t rc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) rc[u] = a.rec[p + u * BLOCK < p1 ? p + u * BLOCK : p1 - 1];  // unconditional loads overlap
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p + u * BLOCK >= p1) break;
            uint64_t slots = rc[u] >> kRowBucketBits;
            if (slots == kRunField) {
                const uint32_t k = a.roff[p + u * BLOCK];
                slots = (uint64_t)run_slots(a.brp[k + 1] - a.brp[k], a.align);
            }
            atomicAdd(&s_cnt[rc[u] & (kRowBucketRows - 1)], (unsigned long long)slots);
        }
    }
    __syncthreads();
    const int64_t r0 = b << kRowBucketBits;
    for (int i = threadIdx.x; i < kRowBucketRows && r0 + i < m; i += BLOCK) a.rowflop[r0 + i] = s_cnt[i];
}

// Pass 3, fixed order: the same per-row totals, but a run's offset in its
// row is the sum of the slots of the row's runs from earlier entries of A
// (A is column-major, so earlier entries of one row are earlier columns),
// whatever order the scatter left the records in.  The bucket's records
// with at least one slot are first grouped by row (a counting sort into
// lste/lsts/lstp over the bucket's own record range); each then adds up the
// slots of its row's records with a smaller entry index.  A row is at most
// det_tmax slots, so it has at most that many such records; a wider row
// is skipped (the plan is then refused).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_bucket_count_det(RowBucketArgs a, int64_t m) {
    constexpr int RPT = kRowBucketRows / BLOCK;
    static_assert(kRowBucketRows % BLOCK == 0, "whole rows per thread");
    __shared__ unsigned long long s_cnt[kRowBucketRows];
    __shared__ uint32_t s_n[kRowBucketRows];      // records per row (fill cursors in between)
    __shared__ uint32_t s_start[kRowBucketRows];  // the row's first record in the grouped lists
    __shared__ uint64_t s_red[BLOCK / kWave];
    __shared__ uint64_t s_scan[BLOCK / kWave + 1];
    for (int i = threadIdx.x; i < kRowBucketRows; i += BLOCK) {
        s_cnt[i] = 0;
        s_n[i] = 0;
    }
    const int64_t b = blockIdx.x;
    if (b == 0) {
        uint64_t f = 0;
        for (int g = threadIdx.x; g < a.ngrp; g += BLOCK) f += a.gflop[g];
        f = block_sum<BLOCK>(f, s_red);
        if (threadIdx.x == 0) a.info->flop = f;
    }
    __syncthreads();
    const uint32_t p0 = a.hist[b * a.ngrp], p1 = a.hist[(b + 1) * a.ngrp];
    auto slots_of = [&](uint32_t p, uint32_t rc) -> uint64_t {
        uint64_t sl = rc >> kRowBucketBits;
        if (sl == kRunField) {
            const uint32_t k = a.roff[p];
            sl = (uint64_t)run_slots(a.brp[k + 1] - a.brp[k], a.align);
        }
        return sl;
    };
    for (int64_t pp = (int64_t)p0 + threadIdx.x; pp < p1; pp += BLOCK) {
        const uint32_t p = (uint32_t)pp;
        const uint32_t rc = a.rec[p];
        const uint32_t row = rc & (kRowBucketRows - 1);
        const uint64_t sl = slots_of(p, rc);
        if (sl) {
            atomicAdd(&s_cnt[row], (unsigned long long)sl);
            atomicAdd(&s_n[row], 1u);
        }
    }
    __syncthreads();
    uint32_t listed;
    {
        uint32_t c[RPT];
        uint64_t t = 0;
#pragma unroll
        for (int x = 0; x < RPT; ++x) {
            c[x] = s_n[threadIdx.x * RPT + x];
            t += c[x];
        }
        uint64_t total;
        uint64_t ex = block_excl_scan<BLOCK, SumOp>(t, s_scan, total);
        listed = (uint32_t)total;
#pragma unroll
        for (int x = 0; x < RPT; ++x) {
            s_start[threadIdx.x * RPT + x] = (uint32_t)ex;
            s_n[threadIdx.x * RPT + x] = 0;
            ex += c[x];
        }
    }
    __syncthreads();
    for (int64_t pp = (int64_t)p0 + threadIdx.x; pp < p1; pp += BLOCK) {
        const uint32_t p = (uint32_t)pp;
        const uint32_t rc = a.rec[p];
        const uint32_t row = rc & (kRowBucketRows - 1);
        const uint64_t sl = slots_of(p, rc);
        if (sl) {
            const uint32_t q = p0 + s_start[row] + atomicAdd(&s_n[row], 1u);
            a.lste[q] = a.recent[p];
            a.lsts[q] = (uint32_t)sl;
            a.lstp[q] = p;
        } else {
            a.roff[p] = 0;  // a run of no tuples
        }
    }
    __syncthreads();
    for (int64_t qq = (int64_t)p0 + threadIdx.x; qq < (int64_t)p0 + listed; qq += BLOCK) {
        const uint32_t q = (uint32_t)qq;
        const uint32_t p = a.lstp[q];
        const uint32_t row = a.rec[p] & (kRowBucketRows - 1);
        if (s_cnt[row] > (unsigned long long)a.det_tmax) continue;  // a wide row: refused after the step
        const uint32_t e = a.lste[q];
        const uint32_t l0 = p0 + s_start[row], l1 = l0 + s_n[row];
        uint64_t off = 0;
        for (uint32_t x = l0; x < l1; ++x) off += a.lste[x] < e ? a.lsts[x] : 0u;
        a.roff[p] = (uint32_t)off;
    }
    __syncthreads();
    const int64_t r0 = b << kRowBucketBits;
    for (int i = threadIdx.x; i < kRowBucketRows && r0 + i < m; i += BLOCK) a.rowflop[r0 + i] = s_cnt[i];
}

// Pass 4 (after the row scan and the bin cut): one workgroup per bucket
// places every record's run inside its bin.  The runs of a bin are not
// grouped by row (the sort orders the bin anyway): the part of a bin inside
// the bucket (its rows there, a "segment") is filled by one LDS cursor in
// record order, which follows the entry order of A and so the column order
// the expand runs in.  Runs that are neighbours in memory are then written
// close together in time, and a bin has one partly written line of keys
// and one of values at a time instead of one per row, so far fewer partial
// lines leave the caches (ER n=2^20, d=16: expand 2.13 -> 2.01 ms).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_bucket_dest(RowBucketArgs a, int64_t m) {
    __shared__ uint64_t s_base[kRowBucketRows];          // per row: its slot range's first slot
    __shared__ unsigned long long s_cur[kRowBucketRows];  // per segment (by its first row): fill cursor
    __shared__ uint32_t s_rl[kRowBucketRows];
    __shared__ uint16_t s_first[kRowBucketRows];          // per row: its segment's first row in the bucket
    const int64_t b = blockIdx.x;
    const int64_t r0 = b << kRowBucketBits;
    for (int i = threadIdx.x; i < kRowBucketRows; i += BLOCK) {
        s_cur[i] = 0;
        if (r0 + i < m) {
            const RowTab rt = a.rowtab[r0 + i];
            s_base[i] = (uint64_t)rt.base;
            s_rl[i] = rt.rl;
            s_first[i] = (uint16_t)((uint32_t)i > rt.rl ? (uint32_t)i - rt.rl : 0u);
        }
    }
    __syncthreads();
    const uint32_t p0 = a.hist[b * a.ngrp], p1 = a.hist[(b + 1) * a.ngrp];
    constexpr int U = 4;
    for (int64_t p = (int64_t)p0 + threadIdx.x; p < p1; p += (int64_t)BLOCK * U) {
        uint32_t rc[U], kk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = p + u * BLOCK < p1 ? p + u * BLOCK : p1 - 1;  // unconditional loads overlap
            rc[u] = a.rec[q];
            kk[u] = a.roff[q];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p + u * BLOCK >= p1) break;
            const uint32_t row = rc[u] & (kRowBucketRows - 1);
            uint64_t slots = rc[u] >> kRowBucketBits;
            if (slots == kRunField) slots = (uint64_t)run_slots(a.brp[kk[u] + 1] - a.brp[kk[u]], a.align);
            const uint32_t f = s_first[row];
            const uint64_t off = atomicAdd(&s_cur[f], (unsigned long long)slots);
            a.entrec[p + u * BLOCK] = ent_pack(s_base[f] + off, s_rl[row]);
        }
    }
}

// Pass 4 of the fixed summation order: runs stay grouped by row, each at
// the offset k_bucket_count_det gave it (the workgroups of a bucket take
// gridDim.y slices of its records; the bucket's rows' first slots and
// rows-in-bin are held in LDS).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_bucket_dest_rows(RowBucketArgs a, int64_t m) {
    __shared__ uint64_t s_base[kRowBucketRows];
    __shared__ uint32_t s_rl[kRowBucketRows];
    const int64_t b = blockIdx.x;
    const int64_t r0 = b << kRowBucketBits;
    for (int i = threadIdx.x; i < kRowBucketRows; i += BLOCK) {
        if (r0 + i < m) {
            const RowTab rt = a.rowtab[r0 + i];
            s_base[i] = (uint64_t)rt.base;
            s_rl[i] = rt.rl;
        }
    }
    __syncthreads();
    const uint32_t q0 = a.hist[b * a.ngrp], q1 = a.hist[(b + 1) * a.ngrp];
    const uint32_t per = (q1 - q0 + gridDim.y - 1) / gridDim.y;
    const uint32_t p0 = q0 + per * blockIdx.y;
    const uint32_t p1 = p0 + per < q1 ? p0 + per : q1;
    constexpr int U = 4;
    for (int64_t p = (int64_t)p0 + threadIdx.x; p < p1; p += (int64_t)BLOCK * U) {
        uint32_t rc[U], off[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t q = p + u * BLOCK < p1 ? p + u * BLOCK : p1 - 1;  // unconditional loads overlap
            rc[u] = a.rec[q];
            off[u] = a.roff[q];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p + u * BLOCK >= p1) break;
            const uint32_t row = rc[u] & (kRowBucketRows - 1);
            a.entrec[p + u * BLOCK] = ent_pack(s_base[row] + off[u], s_rl[row]);
        }
    }
}

// Pass 5: each entry's run destination from its record.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_bucket_offsets(RowBucketArgs a) {
    const int64_t e0 = blockIdx.x * a.epw;
    const int64_t e1 = e0 + a.epw < a.nnz ? e0 + a.epw : a.nnz;
    constexpr int U = 4;
    for (int64_t e = e0 + threadIdx.x; e < e1; e += (int64_t)BLOCK * U) {
        uint32_t ps[U];
#pragma unroll
        for (int u = 0; u < U; ++u) ps[u] = e + u * BLOCK < e1 ? a.posof[e + u * BLOCK] : 0u;
        uint64_t d[U];
#pragma unroll
        for (int u = 0; u < U; ++u) d[u] = a.entrec[ps[u]];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e + u * BLOCK < e1) a.ent[e + u * BLOCK] = d[u];
    }
}

// Run destinations when the run offsets came from device atomics (k_rowflop):
// one thread per entry of A, its row's facts gathered from the row table.
__global__ __launch_bounds__(256) void k_entry_dest(int64_t nnz, const int32_t *ari, const uint32_t *runpos,
                                                    const RowTab *rowtab, uint64_t *ent);

// Exclusive scan of the bucket-major histogram, in place (total at [n]).
struct HistSrc {
    const uint32_t *h;
    __device__ uint64_t operator()(int64_t i) const { return h[i]; }
};
struct HistDst : NoSide {
    uint32_t *h;
    int64_t n;
    __device__ void operator()(int64_t i, uint64_t excl, uint64_t) const { h[i] = (uint32_t)excl; }
    __device__ void total(uint64_t t) const { h[n] = (uint32_t)t; }
};

// R = exclusive scan of rowflop (in place); side: largest row flop <= T/2.
struct RowFlopSrc {
    const uint64_t *rf;
    __device__ uint64_t operator()(int64_t r) const { return rf[r]; }
};
struct RowFlopDst {
    uint64_t *R;
    int64_t m;
    uint64_t thalf;
    SymInfo *info;
    __device__ void operator()(int64_t r, uint64_t excl, uint64_t) const { R[r] = excl; }
    __device__ void total(uint64_t t) const { R[m] = t; }
    __device__ uint64_t side(int64_t, uint64_t e) const { return e <= thalf ? e : 0; }
    __device__ void side_commit(uint64_t v) const { atomic_max_agent(&info->maxnormal, v); }
};

// Bin cut.  With H = T - maxnormal, cap = 2^min(rowbits, 24) - 1 and row weight
// g(r) = R[r] + c*r (c = ceil(H / cap) >= 1), a row starts a new bin when it
// is the first row, when it or its predecessor is big (row flop > T/2), or
// when floor(g/H) differs from its predecessor's.  Rows s..e of one bin of
// normal rows have g(e) - g(s) <= H - 1 and g(e) - g(s) >= c*(e - s), so the
// bin holds <= H - 1 + maxnormal < T tuples and e - s + 1 <= cap rows; a big
// row is a bin by itself.  The row part of a key is then at most
// 2^rowbits - 2, so no real key equals the all-ones sentinel, even at
// column 2^colbits - 1.  Payload: (count of starts) << 31 | last start row.
struct BinOp {
    static __device__ __forceinline__ uint64_t identity() { return 0; }
    static __device__ __forceinline__ uint64_t combine(uint64_t a, uint64_t b) {
        const uint64_t cb = b >> 31;
        return (((a >> 31) + cb) << 31) | (cb ? (b & 0x7fffffffull) : (a & 0x7fffffffull));
    }
};
struct BinSrc {
    const uint64_t *R;
    const SymInfo *info;
    uint64_t T;
    int rowbits;
    const int64_t *prob_row0;  // batched: sorted first rows of the problems (or null)
    int64_t nprob;
    int seg_log;               // >= 0: a bin also starts at every multiple of 2^seg_log
    __device__ uint64_t operator()(int64_t r) const {
        const uint64_t thalf = T / 2;
        const uint64_t H = T - info->maxnormal;
        const int cbits = rowbits < kMaxBinRowBits ? rowbits : kMaxBinRowBits;
        const uint64_t cap = (1ull << cbits) - 1;
        uint64_t c = (H + cap - 1) / cap;
        c = c < 1 ? 1 : c;
        bool start = (r == 0);
        if (!start) {
            const uint64_t rf = R[r + 1] - R[r];
            const uint64_t rfp = R[r] - R[r - 1];
            if (rf > thalf || rfp > thalf) {
                start = true;
            } else {
                const uint64_t g = R[r] + c * (uint64_t)r;
                const uint64_t gp = R[r - 1] + c * (uint64_t)(r - 1);
                start = (g / H) != (gp / H);
            }
            if (!start && prob_row0) {
                int64_t j = last_le(prob_row0, 0, nprob, (int64_t)r);
                start = prob_row0[j] == r;
            }
            if (!start && seg_log >= 0) start = (r & ((1ll << seg_log) - 1)) == 0;
        }
        return start ? ((1ull << 31) | (uint64_t)r) : 0;
    }
};

__global__ __launch_bounds__(256) void k_entry_dest(int64_t nnz, const int32_t *ari, const uint32_t *runpos,
                                                    const RowTab *rowtab, uint64_t *ent) {
    const int64_t e = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (e >= nnz) return;
    const RowTab rt = rowtab[ari[e]];
    ent[e] = ent_pack((uint64_t)rt.base + runpos[e], rt.rl);
}

struct BinDst {
    RowTab *rowtab;
    int32_t *binrow0;
    int64_t *binoff;
    const uint64_t *R;
    int64_t m;
    uint64_t T;
    SymInfo *info;
    int32_t *oversize;  // rows with more than T tuples are listed here (or only counted)
    __device__ void operator()(int64_t r, uint64_t excl, uint64_t e) const {
        const uint64_t incl = BinOp::combine(excl, e);
        const uint64_t bin = (incl >> 31) - 1;
        const uint64_t l = incl & 0x7fffffffull;
        RowTab rt;
        rt.base = (int64_t)R[r];
        rt.rl = (uint32_t)(r - (int64_t)l);
        rt.bin = (uint32_t)bin;
        rowtab[r] = rt;
        if (e) {
            binrow0[bin] = (int32_t)r;
            binoff[bin] = (int64_t)R[r];
            if (R[r + 1] - R[r] > T) {
                const uint64_t slot = atomic_add_agent(&info->noversize, (uint64_t)1);
                if (oversize) oversize[slot] = (int32_t)r;
            }
        }
    }
    __device__ void total(uint64_t t) const {
        const uint64_t nb = t >> 31;
        binrow0[nb] = (int32_t)m;
        binoff[nb] = (int64_t)R[m];
        info->nbins = nb;
    }
    __device__ uint64_t side(int64_t r, uint64_t) const { return R[r + 1] - R[r]; }
    __device__ void side_commit(uint64_t v) const { atomic_max_agent(&info->maxrow, v); }
};

// info->maxbin = the most tuple slots of any bin (bins < info->nbins).  A
// grid-stride loop and one atomic per workgroup.
__global__ __launch_bounds__(256) void k_bin_max(const int64_t *binoff, int64_t maxbins, SymInfo *info) {
    __shared__ uint64_t s_max[256 / kWave];
    const int64_t nb = (int64_t)info->nbins < maxbins ? (int64_t)info->nbins : maxbins;
    uint64_t v = 0;
    for (int64_t b = blockIdx.x * (int64_t)256 + threadIdx.x; b < nb; b += (int64_t)gridDim.x * 256) {
        const uint64_t sz = (uint64_t)(binoff[b + 1] - binoff[b]);
        v = sz > v ? sz : v;
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const uint64_t o = __shfl_xor(v, d, kWave);
        v = o > v ? o : v;
    }
    if (lane_id() == 0) s_max[threadIdx.x / kWave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 256 / kWave; ++i) v = s_max[i] > v ? s_max[i] : v;
        if (v) atomic_max_agent(&info->maxbin, v);
    }
}

// kstart[c] = column holding tuple c*C (c < nchunks); kstart[nchunks] = K-1.
__global__ void k_chunk_start(int64_t nchunks, int64_t C, int64_t K, const int64_t *F, int32_t *kstart) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c > nchunks) return;
    if (c == nchunks) {
        kstart[c] = (int32_t)(K - 1);
        return;
    }
    kstart[c] = (int32_t)last_le(F, 0, K, c * C);
}

// ---------------------------------------------------------------------------
// Expand (Algorithm 2's outer-product loop).  The slot space [0, slots) is
// cut into chunks of W slots, one wave each; slot t lies in column k of A /
// row k of B with F[k] <= t < F[k+1] (F: scan of the columns' slots), and is
// the product of the i-th entry of A(:,k) and the j-th entry of B(k,:),
// (i, j) = divmod(t - F[k], run slots of B(k,:)); slots with j past
// nnz(B(k,:)) are run padding and get the sentinel key.  The tuples of one
// A entry e = (r, k) form a run that goes to the slots of r's bin, at the
// place ent[e] the symbolic step fixed, so every bin is one contiguous slot
// range and no append needs an atomic.
// Consecutive lanes take consecutive tuples, so each run is written by
// consecutive lanes to consecutive addresses.
struct ExpandArgs {
    int64_t flop, K;
    const int64_t *F;
    const int32_t *kstart;
    const int64_t *acp;
    const double *av;
    const int64_t *brp;
    const int32_t *bci;
    const double *bv;
    const uint64_t *ent;     // per A entry: its run's first slot and row in bin (ent_pack)
    uint32_t *keys;
    void *vals;
    int cb;
    uint32_t *err;
    const int64_t *astart;  // rounds: first entry of A(:,k) in the round's rows (null: all of A(:,k))
    int64_t slot0;          // rounds: slot of the round's first tuple
    int align;              // run alignment in slots
};

// (q, r) = divmod(x, d) for 0 <= x, 1 <= d; float reciprocal with an exact
// integer correction when x < 2^24, integer division otherwise.
__device__ __forceinline__ void divmod_u(int64_t x, int64_t d, int64_t &q, int64_t &r) {
    if (x < (1 << 24) && d < (1 << 24)) {
        int32_t qq = (int32_t)((float)x * __builtin_amdgcn_rcpf((float)d));
        int32_t rr = (int32_t)x - qq * (int32_t)d;
        while (rr < 0) {
            --qq;
            rr += (int32_t)d;
        }
        while (rr >= (int32_t)d) {
            ++qq;
            rr -= (int32_t)d;
        }
        q = qq;
        r = rr;
    } else if (x < 0x100000000ll && d < 0x100000000ll) {
        const uint32_t qq = (uint32_t)x / (uint32_t)d;
        q = qq;
        r = x - (int64_t)qq * d;
    } else {
        q = x / d;
        r = x - q * d;
    }
}

// Chunks that span many short columns: each lane finds its own column.  The
// wave holds the facts of 64 consecutive columns, one per lane (where the
// column's tuples start in the flop space, B's row, A's column start), and
// takes 64 consecutive tuples per step; a lane's column is the last one
// starting at or before its tuple (a binary search over the lanes), and its
// (A entry, B entry) pair comes from a divmod by the column's run slots.
constexpr int kShortCols = 8;  // a chunk spanning more columns takes this path

template <int W, class VT>
__device__ __forceinline__ void expand_lanes(const int64_t *__restrict__ F, const int64_t *__restrict__ acp,
                                             const int64_t *__restrict__ astart, const int64_t *__restrict__ brp,
                                             const uint64_t *__restrict__ ent, const double *__restrict__ avv,
                                             const int32_t *__restrict__ bci, const double *__restrict__ bvals,
                                             const TupleArr<VT> tup, uint32_t *__restrict__ err, int cb,
                                             int64_t flop, int64_t slot0, int align, int64_t K, int64_t kb, int64_t t,
                                             const int64_t t1) {
    const int lane = (int)lane_id();
    bool bad = false;
    while (t < t1) {
        const int64_t kk = kb + lane;
        int64_t f0 = INT64_MAX;  // past the columns: never owns a tuple
        int64_t as = 0;
        uint32_t bs = 0, nbt = 0;
        if (kk < K) {
            f0 = F[kk];
            const int64_t b0 = brp[kk];
            bs = (uint32_t)b0;
            nbt = (uint32_t)(brp[kk + 1] - b0);
            as = astart ? astart[kk] : acp[kk];
        }
        const int64_t kn = kb + kWave;
        const int64_t wend0 = F[kn < K ? kn : K];  // where the next window's first column starts
        const int64_t wend = wend0 < t1 ? wend0 : t1;
        constexpr int U = 4;
        for (int64_t tt = t; tt < wend; tt += U * kWave) {
            int64_t ii[U], asu[U];
            uint32_t jj[U], nbu[U], bsu[U];
            bool on[U], own[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t ts = tt + u * kWave;  // the step's first tuple (wave-uniform)
                const int64_t d = f0 - ts;
                const int rel = d < -1 ? -1 : (d > kWave ? kWave : (int)d);
                int L = 0;
#pragma unroll
                for (int s = kWave / 2; s >= 1; s >>= 1)
                    if (__shfl(rel, L + s, kWave) <= lane) L += s;
                const int64_t fL = __shfl(f0, L, kWave);
                nbu[u] = __shfl(nbt, L, kWave);
                bsu[u] = __shfl(bs, L, kWave);
                asu[u] = __shfl(as, L, kWave);
                on[u] = ts + lane < wend;
                own[u] = on[u] && fL <= ts + lane && nbu[u] > 0;
                int64_t q = 0, r = 0;
                if (own[u]) divmod_u(ts + lane - fL, run_slots(nbu[u], align), q, r);
                ii[u] = q;
                jj[u] = (uint32_t)r;
            }
            uint64_t en[U];
            uint32_t col[U];
            double av[U], bvv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t e = own[u] ? asu[u] + ii[u] : 0;
                // padding slots read the run's last B entry
                const uint32_t jb = own[u] ? (jj[u] < nbu[u] ? jj[u] : nbu[u] - 1u) : 0u;
                const uint32_t bi = own[u] ? bsu[u] + jb : 0u;
                en[u] = ent[e];
                av[u] = avv[e];
                col[u] = (uint32_t)bci[bi];
                bvv[u] = bvals[bi];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!on[u]) continue;
                if (!own[u]) {
                    bad = true;
                    continue;
                }
                const int64_t slot = (int64_t)(en[u] & kEntSlotMask) - slot0 + jj[u];
                const bool real = jj[u] < nbu[u];
                const uint32_t rl = (uint32_t)(en[u] >> kEntSlotBits);
                if ((uint64_t)slot < (uint64_t)flop) {
                    tup.put(slot, real ? ((rl << cb) | col[u]) : kSentinel, real ? (VT)(av[u] * bvv[u]) : (VT)0);
                } else {
                    bad = true;
                }
            }
        }
        if (wend > t) t = wend;
        kb = kn;
    }
    if (bad) atomic_or_agent(err, (uint32_t)kErrBinOverflow);
}

// Chunks that span at most kShortCols + 1 columns, software-pipelined: the
// wave takes its chunk in groups of U 64-tuple steps and issues the loads of
// the next group before the stores of the current one.  Vector loads and
// stores share one in-order completion counter, so a wave that waited for a
// load issued after its stores would also wait for those stores; issued the
// other way round, the stores of one group stay in flight while the wave
// waits for the next group's operands.  Each lane finds its tuple's column
// among the chunk's columns (their starts relative to the chunk sit in
// scalar registers), then (A entry, B entry) = divmod(offset in the column,
// run slots of B's row); a slot past nnz(B(k,:)) is run padding.
template <class VT, int U>
struct ExpandGroup {
    uint64_t en[U];
    double av[U], bv[U];
    uint32_t col[U], j[U], nb[U];
    bool on[U];
};

template <int W, class VT>
__device__ __forceinline__ void expand_flat(const int64_t *__restrict__ F, const int64_t *__restrict__ acp,
                                            const int64_t *__restrict__ astart, const int64_t *__restrict__ brp,
                                            const uint64_t *__restrict__ ent, const double *__restrict__ avv,
                                            const int32_t *__restrict__ bci, const double *__restrict__ bvals,
                                            const TupleArr<VT> tup, uint32_t *__restrict__ err, int cb,
                                            int64_t flop, int64_t slot0, int align, int64_t kb, int nc, int64_t t0,
                                            int64_t t1) {
    constexpr int U = 2;
    constexpr int GS = U * kWave;  // tuples per group
    const int lane = (int)lane_id();
    // one column per lane: where its slots start, B's row, A's column
    int64_t fF = 0, fA = 0, fB = 0;
    int32_t fN = 0;
    int32_t rel = W;  // column start relative to t0, clamped to [-1, W]
    if (lane < nc) {
        const int64_t k = kb + lane;
        fF = F[k];
        fB = brp[k];
        fN = (int32_t)(brp[k + 1] - fB);
        fA = astart ? astart[k] : acp[k];
        const int64_t d = fF - t0;
        rel = d < -1 ? -1 : (d > W ? W : (int32_t)d);
    }
    int32_t rs[kShortCols + 1];
#pragma unroll
    for (int l = 0; l <= kShortCols; ++l) rs[l] = __builtin_amdgcn_readlane(rel, l);
    const int last = (int)(t1 - 1 - t0);
    bool bad = false;
    auto issue = [&](int g, ExpandGroup<VT, U> &G) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int o = g * GS + u * kWave + lane;
            G.on[u] = o <= last;
            const int oc = o <= last ? o : last;  // lanes past the end load the last tuple's operands
            int c = 0;
#pragma unroll
            for (int l = 1; l <= kShortCols; ++l) c += rs[l] <= oc ? 1 : 0;
            const int64_t Fc = __shfl(fF, c, kWave);
            const int64_t Bc = __shfl(fB, c, kWave);
            const int64_t Ac = __shfl(fA, c, kWave);
            const uint32_t Nc = (uint32_t)__shfl(fN, c, kWave);
            int64_t i = 0, j = 0;
            if (Nc > 0) divmod_u(t0 + oc - Fc, run_slots(Nc, align), i, j);
            const uint32_t jb = (uint32_t)j < Nc ? (uint32_t)j : Nc - 1u;  // padding reads the run's last B entry
            const int64_t e = Nc > 0 ? Ac + i : 0;
            const int64_t bi = Nc > 0 ? Bc + jb : 0;
            G.en[u] = ent[e];
            G.av[u] = avv[e];
            G.col[u] = (uint32_t)bci[bi];
            G.bv[u] = bvals[bi];
            G.j[u] = (uint32_t)j;
            G.nb[u] = Nc;
        }
    };
    auto finish = [&](const ExpandGroup<VT, U> &G) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!G.on[u]) continue;
            if (G.nb[u] == 0) {  // no column of the chunk holds this slot: a broken plan
                bad = true;
                continue;
            }
            const int64_t slot = (int64_t)(G.en[u] & kEntSlotMask) - slot0 + G.j[u];
            const bool real = G.j[u] < G.nb[u];
            const uint32_t key = real ? (((uint32_t)(G.en[u] >> kEntSlotBits) << cb) | G.col[u]) : kSentinel;
            if ((uint64_t)slot < (uint64_t)flop) tup.put(slot, key, real ? (VT)(G.av[u] * G.bv[u]) : (VT)0);
            else bad = true;
        }
    };
    const int ng = (int)((t1 - t0 + GS - 1) / GS);
    ExpandGroup<VT, U> ga, gb;
    issue(0, ga);
    for (int g = 0; g < ng; g += 2) {
        if (g + 1 < ng) issue(g + 1, gb);
        finish(ga);
        if (g + 1 >= ng) break;
        if (g + 2 < ng) issue(g + 2, ga);
        finish(gb);
    }
    if (bad) atomic_or_agent(err, (uint32_t)kErrBinOverflow);
}

// A chunk inside one column (long columns: hub rows of B times long columns
// of A).  The column's facts are wave-uniform and each lane's (A entry,
// B entry) pair advances by (64 div s, 64 mod s) per step with a carry (s:
// the run's slots), so only the first step divides; the groups are
// pipelined as in expand_flat.
template <int W, class VT>
__device__ __forceinline__ void expand_column(const int64_t *__restrict__ F, const int64_t *__restrict__ acp,
                                              const int64_t *__restrict__ astart, const int64_t *__restrict__ brp,
                                              const uint64_t *__restrict__ ent, const double *__restrict__ avv,
                                              const int32_t *__restrict__ bci, const double *__restrict__ bvals,
                                              const TupleArr<VT> tup, uint32_t *__restrict__ err, int cb,
                                              int64_t flop, int64_t slot0, int align, int64_t k, int64_t t0,
                                              int64_t t1) {
    constexpr int U = 2;
    constexpr int GS = U * kWave;
    const uint32_t lane = lane_id();
    const int64_t Fk = F[k];
    const int64_t bs = brp[k];
    const uint32_t nbt = (uint32_t)(brp[k + 1] - bs);  // B entries of the run
    if (nbt == 0) {  // no tuple can lie in this column: a broken plan
        if (lane == 0) atomic_or_agent(err, (uint32_t)kErrBinOverflow);
        return;
    }
    const uint32_t nbu = (uint32_t)run_slots(nbt, align);  // its slots
    const int64_t as = astart ? astart[k] : acp[k];
    const uint64_t *enk = ent + as;
    const double *avk = avv + as;
    const int32_t *bck = bci + bs;
    const double *bvk = bvals + bs;
    int64_t i0, j0, il, jl;
    divmod_u(t0 - Fk + lane, nbu, i0, j0);
    divmod_u(t1 - 1 - Fk, nbu, il, jl);  // the chunk's last tuple: lanes past the end load its operands
    uint32_t ii = (uint32_t)i0, jj = (uint32_t)j0;
    const uint32_t di = nbu > kWave ? 0u : (uint32_t)kWave / nbu;
    const uint32_t dj = nbu > kWave ? (uint32_t)kWave : (uint32_t)kWave - di * nbu;
    const int last = (int)(t1 - 1 - t0);
    bool bad = false;
    auto issue = [&](int g, ExpandGroup<VT, U> &G) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int o = g * GS + u * kWave + (int)lane;
            G.on[u] = o <= last;
            const uint32_t iu = G.on[u] ? ii : (uint32_t)il;
            const uint32_t ju = G.on[u] ? jj : (uint32_t)jl;
            ii += di;
            jj += dj;
            if (jj >= nbu) {
                jj -= nbu;
                ++ii;
            }
            const uint32_t jb = ju < nbt ? ju : nbt - 1u;  // padding reads the run's last B entry
            G.en[u] = enk[iu];
            G.av[u] = avk[iu];
            G.col[u] = (uint32_t)bck[jb];
            G.bv[u] = bvk[jb];
            G.j[u] = ju;
            G.nb[u] = nbt;
        }
    };
    auto finish = [&](const ExpandGroup<VT, U> &G) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!G.on[u]) continue;
            const int64_t slot = (int64_t)(G.en[u] & kEntSlotMask) - slot0 + G.j[u];
            const bool real = G.j[u] < G.nb[u];
            const uint32_t key = real ? (((uint32_t)(G.en[u] >> kEntSlotBits) << cb) | G.col[u]) : kSentinel;
            if ((uint64_t)slot < (uint64_t)flop) tup.put(slot, key, real ? (VT)(G.av[u] * G.bv[u]) : (VT)0);
            else bad = true;
        }
    };
    const int ng = (int)((t1 - t0 + GS - 1) / GS);
    ExpandGroup<VT, U> ga, gb;
    issue(0, ga);
    for (int g = 0; g < ng; g += 2) {
        if (g + 1 < ng) issue(g + 1, gb);
        finish(ga);
        if (g + 1 >= ng) break;
        if (g + 2 < ng) issue(g + 2, ga);
        finish(gb);
    }
    if (bad) atomic_or_agent(err, (uint32_t)kErrBinOverflow);
}

// One wave per chunk of W tuples: a chunk inside one column takes
// expand_column, over at most kShortCols + 1 columns expand_flat, over more
// (short columns: AMG, small d) expand_lanes.  The body takes every array as a restrict pointer: the
// arrays it reads are never written by it, so loads need not wait for
// earlier stores.
template <int W, class VT>
__device__ __forceinline__ void expand_body(const int64_t *__restrict__ F, const int32_t *__restrict__ kstart,
                                            const int64_t *__restrict__ acp, const int64_t *__restrict__ astart,
                                            const int64_t *__restrict__ brp, const uint64_t *__restrict__ ent,
                                            const double *__restrict__ avv,
                                            const int32_t *__restrict__ bci, const double *__restrict__ bvals,
                                            const TupleArr<VT> tup, uint32_t *__restrict__ err, int cb,
                                            int64_t flop, int64_t slot0, int align, int64_t nchunks, int64_t K) {
    const int64_t wave = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (wave >= nchunks) return;
    const int64_t t0 = wave * (int64_t)W;
    const int64_t t1 = (t0 + W < flop) ? t0 + W : flop;
    const int64_t k = kstart[wave];
    const int64_t nc = kstart[wave + 1] - k + 1;  // columns the chunk touches
    if (nc == 1)
        expand_column<W, VT>(F, acp, astart, brp, ent, avv, bci, bvals, tup, err, cb, flop, slot0, align, k, t0, t1);
    else if (nc > kShortCols + 1)
        expand_lanes<W, VT>(F, acp, astart, brp, ent, avv, bci, bvals, tup, err, cb, flop, slot0, align, K, k, t0,
                            t1);
    else
        expand_flat<W, VT>(F, acp, astart, brp, ent, avv, bci, bvals, tup, err, cb, flop, slot0, align, k, (int)nc,
                           t0, t1);
}

template <int W, class VT>
__global__ __launch_bounds__(256) void k_expand(ExpandArgs a, int64_t nchunks) {
    expand_body<W, VT>(a.F, a.kstart, a.acp, a.astart, a.brp, a.ent, a.av, a.bci, a.bv,
                       TupleArr<VT>(a.keys, a.vals), a.err, a.cb, a.flop, a.slot0, a.align, nchunks, a.K);
}

// ---------------------------------------------------------------------------
// ConvertCSR, part 1: entries per row of C.  A bin's tuples are contiguous
// and carry their row inside the bin in the key, so nnz(C(r,:)) is the
// number of distinct keys with r's row bits.  One workgroup per bin inserts the
// bin's keys into an LDS hash set (open addressing, linear probing); a bin
// of at most 256 rows credits each newly inserted key to its row (one LDS
// add per same-row segment of a wave), a bin of more rows lets each
// occupied slot add one to its key's row once every key is in.  Only keys
// are read.
struct CountArgs {
    const int32_t *binrow0;
    const int64_t *binoff;
    const uint32_t *keys;  // key of slot i at keys[i * kstride]
    int kstride;           // 1: FP64 key array; 2: FP32c {key, value} words
    int cb;
    uint32_t *rownnz;
    uint32_t *err;
    int64_t T;                 // bins with more tuples are wide and done elsewhere
    int64_t bin0;              // first bin of the launch
    int64_t slot0;             // slot of the launch's first tuple in `keys`
    int64_t row_base;          // rownnz is indexed by row - row_base
    const uint64_t *nbins;     // if set, blocks at or past *nbins exit
};

template <int BLOCK, int TMAX>
__global__ __launch_bounds__(BLOCK) void k_row_nnz(CountArgs a) {
    constexpr int TS = 2 * TMAX;  // table slots, load factor <= 1/2
    constexpr int LOG_TS = (TS >= 16384) ? 14 : (TS >= 8192) ? 13 : (TS >= 4096) ? 12 : 11;
    static_assert((1 << LOG_TS) == TS, "table size must be a power of two");
    constexpr uint32_t EMPTY = 0xffffffffu;
    static_assert(TS >= TMAX, "the row counters reuse the table");
    __shared__ uint32_t table[TS];
    uint32_t *rowcnt = table;  // after the table has been read back
    constexpr int kSmallRows = 256;
    __shared__ uint32_t rowcnt_small[kSmallRows];
    if (a.nbins) {
        const uint64_t nb = *a.nbins;
        if (blockIdx.x == 0 && threadIdx.x == 0 && nb > gridDim.x) atomic_or_agent(a.err, (uint32_t)kErrGrid);
        if ((uint64_t)blockIdx.x >= nb) return;
    }
    const int64_t b = a.bin0 + blockIdx.x;
    const int64_t row0 = a.binrow0[b];
    const int nrows = (int)(a.binrow0[b + 1] - row0);
    const int64_t toff = a.binoff[b] - a.slot0;
    const int64_t N64 = a.binoff[b + 1] - a.binoff[b];
    if (N64 > a.T) return;
    int N = (int)N64;
    if (N > TMAX || nrows > TMAX) {
        if (threadIdx.x == 0) atomic_or_agent(a.err, (uint32_t)kErrTile);
        return;
    }
    if (N == 0) {  // rows without tuples
        for (int x = threadIdx.x; x < nrows; x += BLOCK) a.rownnz[row0 - a.row_base + x] = 0;
        return;
    }
    const int ks = a.kstride;
    const uint32_t *gk = a.keys + toff * ks;
    const int cb = a.cb;
    constexpr int IPT = TMAX / BLOCK;
    uint32_t kr[IPT];
    // all loads first (unconditional: the last key stands in past the end),
    // so their latencies overlap each other and the table's clearing
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int p = i * BLOCK + threadIdx.x;
        kr[i] = gk[(int64_t)(p < N ? p : N - 1) * ks];
    }
    for (int x = threadIdx.x; x < TS; x += BLOCK) table[x] = EMPTY;
    const bool small = nrows <= kSmallRows;
    if (small)
        for (int x = threadIdx.x; x < nrows; x += BLOCK) rowcnt_small[x] = 0;
    __syncthreads();
    uint32_t fresh = 0;  // bit i: key i entered the set by this thread's swap
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const uint32_t key = kr[i];
        const int p = i * BLOCK + threadIdx.x;
        if (p < N && key != kSentinel) {  // padding slots hold the sentinel (== EMPTY)
            uint32_t h = (key * 0x9E3779B1u) >> (32 - LOG_TS);
            while (true) {
                const uint32_t old = atomicCAS(&table[h], EMPTY, key);
                if (old == EMPTY) fresh |= 1u << i;
                if (old == EMPTY || old == key) break;
                h = (h + 1) & (TS - 1);
            }
        }
    }
    if (small) {
        // Bins of at most kSmallRows rows: each key that entered the set
        // (exactly one lane per distinct key) counts for its row.  A wave's
        // consecutive lanes hold consecutive tuples, mostly of one run (one
        // row), so each segment of lanes with the same row adds its new
        // keys to the row with one LDS update, after every lane's inserts
        // are done (the wave is converged here).
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int p = i * BLOCK + threadIdx.x;
            const bool real = p < N && kr[i] != kSentinel;
            const uint32_t row = real ? (cb < 32 ? (kr[i] >> cb) : 0u) : 0xffffffffu;
            const uint64_t fm = ballot(((fresh >> i) & 1u) != 0);
            const uint32_t lane = lane_id();
            const uint32_t prev = __shfl_up(row, 1u, kWave);
            const uint64_t heads = ballot(lane == 0 || prev != row);
            const uint64_t above = heads & ~((2ull << lane) - 1ull);
            const uint32_t end = above ? (uint32_t)__builtin_ctzll(above) : (uint32_t)kWave;
            if (((heads >> lane) & 1ull) && row != 0xffffffffu) {
                const uint64_t seg = (end >= 64u ? ~0ull : ((1ull << end) - 1ull)) & ~((1ull << lane) - 1ull);
                const uint32_t c = (uint32_t)__builtin_popcountll(fm & seg);
                if (c) atomicAdd(&rowcnt_small[row], c);
            }
        }
        __syncthreads();
        for (int x = threadIdx.x; x < nrows; x += BLOCK) a.rownnz[row0 - a.row_base + x] = rowcnt_small[x];
        return;
    }
    __syncthreads();
    // Slots hold the bin's distinct keys in hash order, so neighbouring
    // lanes mostly hit different rows' counters.  The slots are read into
    // registers first; the row counters then take the table's place.
    constexpr int SPT = TS / BLOCK;
    uint32_t slot_key[SPT];
#pragma unroll
    for (int x = 0; x < SPT; ++x) slot_key[x] = table[x * BLOCK + threadIdx.x];
    __syncthreads();
    for (int x = threadIdx.x; x < nrows; x += BLOCK) rowcnt[x] = 0;
    __syncthreads();
#pragma unroll
    for (int x = 0; x < SPT; ++x)
        if (slot_key[x] != EMPTY) atomicAdd(&rowcnt[cb < 32 ? (slot_key[x] >> cb) : 0u], 1u);
    __syncthreads();

    for (int x = threadIdx.x; x < nrows; x += BLOCK) a.rownnz[row0 - a.row_base + x] = rowcnt[x];
}

// rowptr = exclusive scan of the per-row entry counts (rowptr[m] = nnz(C)).
struct RowNnzSrc {
    const uint32_t *rownnz;
    __device__ uint64_t operator()(int64_t r) const { return rownnz[r]; }
};
struct RowPtrDst : NoSide {
    int64_t *rowptr;
    int64_t m;
    const int64_t *base;  // rounds writing one C: entries before the round (or null)
    __device__ int64_t b0() const { return base ? *base : 0; }
    __device__ void operator()(int64_t r, uint64_t excl, uint64_t) const { rowptr[r] = b0() + (int64_t)excl; }
    __device__ void total(uint64_t t) const { rowptr[m] = b0() + (int64_t)t; }
};

// ---------------------------------------------------------------------------
// Batched products.  A batch C_i = A_i * B_i is run as one block-diagonal
// product: A_i's columns and rows and B_i's rows are laid side by side
// (row and inner indices offset, B's column indices kept local because bins
// never span two problems), and every problem's C goes to its own arrays.
struct ProbDesc {
    const int64_t *aptr;
    const int32_t *aidx;
    const double *aval;
    const int64_t *bptr;
    const int32_t *bidx;
    const double *bval;
    int64_t m, k, n, nnza, nnzb;
    int64_t mbase, kbase, abase, bbase;
};
struct OutDesc {
    int64_t *rowptr;
    int32_t *colidx;
    void *val;
    int64_t capacity;
    int64_t row0;  // first row of the problem in the block-diagonal product
    int64_t m;
};

// what: bit 0 = pointers and indices, bit 1 = values.  Problem i = blockIdx.y.
__global__ __launch_bounds__(256) void k_pack(const ProbDesc *pd, int count, int what, int64_t *acp, int32_t *ari,
                                              double *av, int64_t *brp, int32_t *bci, double *bv) {
    const ProbDesc d = pd[blockIdx.y];
    const int64_t stride = (int64_t)gridDim.x * 256;
    const int64_t x0 = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (what & 1) {
        for (int64_t x = x0; x < d.k; x += stride) {
            acp[d.kbase + x] = d.aptr[x] + d.abase;
            brp[d.kbase + x] = d.bptr[x] + d.bbase;
        }
        for (int64_t x = x0; x < d.nnza; x += stride) ari[d.abase + x] = d.aidx[x] + (int32_t)d.mbase;
        for (int64_t x = x0; x < d.nnzb; x += stride) bci[d.bbase + x] = d.bidx[x];
        if ((int)blockIdx.y == count - 1 && x0 == 0) {
            acp[d.kbase + d.k] = d.abase + d.nnza;
            brp[d.kbase + d.k] = d.bbase + d.nnzb;
        }
    }
    if (what & 2) {
        for (int64_t x = x0; x < d.nnza; x += stride) av[d.abase + x] = d.aval[x];
        for (int64_t x = x0; x < d.nnzb; x += stride) bv[d.bbase + x] = d.bval[x];
    }
}

// problem holding global row r (problems sorted by first row; empty
// problems share their successor's first row and are skipped)
__device__ __forceinline__ int prob_of_row(const int64_t *prob_row0, int nprob, int64_t r) {
    return (int)last_le(prob_row0, 0, nprob, r);
}

// Segmented exclusive scan of entries per row, restarting at every
// problem's first row; payload bit 61 = segment start, bits 0..60 = sum.
struct SegSumOp {
    static __device__ __forceinline__ uint64_t identity() { return 0; }
    static __device__ __forceinline__ uint64_t combine(uint64_t a, uint64_t b) {
        constexpr uint64_t F = 1ull << 61;
        return (b & F) ? ((a & F) | b) : (((a | b) & F) | (((a & ~F) + (b & ~F)) & ~F));
    }
};
struct SegRowNnzSrc {
    const uint32_t *rownnz;
    const int64_t *prob_row0;
    int nprob;
    __device__ uint64_t operator()(int64_t r) const {
        const int i = prob_of_row(prob_row0, nprob, r);
        return ((prob_row0[i] == r) ? (1ull << 61) : 0ull) | (uint64_t)rownnz[r];
    }
};
struct SegRowPtrDst : NoSide {
    const OutDesc *outs;
    const int64_t *prob_row0;
    int nprob;
    __device__ void operator()(int64_t r, uint64_t excl, uint64_t e) const {
        constexpr uint64_t F = 1ull << 61;
        const int i = prob_of_row(prob_row0, nprob, r);
        const OutDesc od = outs[i];
        const int64_t before = (e & F) ? 0 : (int64_t)(excl & ~F);
        od.rowptr[r - od.row0] = before;
        if (r - od.row0 == od.m - 1) od.rowptr[od.m] = before + (int64_t)(e & ~F);
    }
    __device__ void total(uint64_t) const {}
};

// ---------------------------------------------------------------------------
// Sort + compress, one workgroup per bin.  The bin's N <= TMAX tuples (a
// contiguous slot range of the tuple array) are loaded once, every load
// issued before the first use; keys are ordered in LDS together with 16-bit
// slot numbers while the values wait in registers; the values are then
// parked in LDS by slot.  Equal keys are summed in sorted order by the first
// tuple of each run (Section 3.5's merge) and written at their final place
// in C.
//
// ConvertCSR (Algorithm 2's last step) is fused in: bins take tickets in
// launch order; once a bin knows how many entries of C it holds (its
// distinct keys), it publishes that count, and a decoupled look-back over
// the earlier bins' counts gives the entries of C before it.  The bin then
// writes its entries and its rows' pointers at their final places.  (The
// virtual rows of wide rows instead get their row pointers from a count
// pass and a scan before the sort: `fused` = 0.)
//
// Repeated keys.  A bin whose keys crowd the sort's buckets first sums
// equal keys in an LDS hash table (in double) and sorts only the distinct
// keys, if at most half of the tile's slots are needed; with given row
// pointers the trigger is at most half as many entries of C as tuples.
//
// Ordering.  Keys are (row in bin) << cb | column.  The default path is a
// one-pass bucket sort: bucket = (key - min) >> s with NB buckets, counted
// and scattered with LDS atomics, after which every key finds its place in
// its (small) bucket by counting the smaller keys there.  Equal keys may
// land in any order: they are summed together, so only rounding changes.
// When a bucket holds more than kBucketLimit keys (clustered columns), the
// bin is ordered instead by a stable LSD radix sort whose per-wave ranks come
// from ballots.
struct SortArgs {
    const int32_t *binrow0;
    const int64_t *binoff;
    const uint32_t *keys;
    const void *vals;
    int cb;
    uint32_t *err;
    int64_t *rowptr;  // single product: C's row pointers, indexed by row - row_base
    int32_t *colidx;
    void *cvals;
    int64_t capacity;
    // batched: per-problem outputs (null for a single product)
    const OutDesc *outs;
    const int64_t *prob_row0;
    int nprob;
    int64_t T;              // bins with more tuples are wide and done elsewhere
    int64_t bin0;           // first bin of the launch
    int64_t slot0;          // slot of the launch's first tuple in `keys` / `vals`
    int64_t row_base;       // rowptr is indexed by row - row_base
    const uint64_t *nbins;  // if set, blocks at or past *nbins exit (unfused only)
    int vshift;             // virtual rows of wide rows: column = (row & vmask) << vshift | key column
    uint32_t vmask;
    // fused ConvertCSR
    int fused;                   // 1: the launch writes C's row pointers itself
    uint32_t *ticket;            // bin order (zeroed)
    uint64_t *status;            // look-back words, one per bin of the launch (zeroed)
    const uint32_t *bignnz;      // rounds: entries of C of each wide row, indexed by row - row_base
    const int64_t *rowptr_base;  // entries of C before the launch's first row (null: none)
    int64_t rows_end;            // single product: one past the launch's last row
    // fixed summation order (k_sort_compress<..., true>): equal keys ordered by
    // slot, each entry of C summed one tuple at a time from its first tuple
    int det;
};

template <class VT>
struct Merge;
template <>
struct Merge<double> {
    // plain double sum
    double s;
    __device__ void zero() { s = 0.0; }
    __device__ void start(double v) { s = v; }
    __device__ void add(double v) { s = s + v; }
    __device__ double result() const { return s; }
};
template <>
struct Merge<float> {
    // Neumaier's compensated sum in float: s + c is the running total
    float s, c;
    __device__ void zero() {
        s = 0.0f;
        c = 0.0f;
    }
    __device__ void start(float v) {
        s = v;
        c = 0.0f;
    }
    __device__ void add(float v) {
        const float t = s + v;
        if (fabsf(s) >= fabsf(v)) c = c + ((s - t) + v);
        else c = c + ((v - t) + s);
        s = t;
    }
    __device__ float result() const { return s + c; }
};
// Sum of two consecutive pieces of a run: x (earlier) then y (later).
__device__ __forceinline__ Merge<double> merge_cat(const Merge<double> &x, const Merge<double> &y) {
    Merge<double> r;
    r.s = x.s + y.s;
    return r;
}
__device__ __forceinline__ Merge<float> merge_cat(const Merge<float> &x, const Merge<float> &y) {
    Merge<float> r = x;
    r.add(y.s);  // compensated add of y's running sum
    r.c = r.c + y.c;
    return r;
}
__device__ __forceinline__ Merge<double> shfl_up_merge(const Merge<double> &x, int d) {
    Merge<double> r;
    r.s = __shfl_up(x.s, (unsigned)d, kWave);
    return r;
}
__device__ __forceinline__ Merge<float> shfl_up_merge(const Merge<float> &x, int d) {
    Merge<float> r;
    r.s = __shfl_up(x.s, (unsigned)d, kWave);
    r.c = __shfl_up(x.c, (unsigned)d, kWave);
    return r;
}

// Loads a bin's N >= 1 tuples (slots [toff, toff + N) of a TupleArr<VT>
// layout) into registers, tuple p = w * 64 * IPT + i * 64 + lane in rk[i],
// rv[i]; past N the key is the sentinel.  Every load is issued before any
// is used: FP64 keys first, so the key phases that follow wait only for them
// while the values are still arriving; FP32c loads each {key, value} word
// once.
template <int BLOCK, int TMAX, class VT>
__device__ __forceinline__ void load_bin(const uint32_t *keys, const void *vals, int64_t toff, int N,
                                         uint32_t (&rk)[TMAX / BLOCK], VT (&rv)[TMAX / BLOCK]) {
    constexpr int IPT = TMAX / BLOCK;
    const int base = (int)(threadIdx.x / kWave) * kWave * IPT + (int)lane_id();
    if constexpr (sizeof(VT) == 8) {
        const uint32_t *gk = keys + toff;
        const VT *gv = (const VT *)vals + toff;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int p = base + i * kWave;
            rk[i] = p < N ? gk[p] : kSentinel;
        }
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int p = base + i * kWave;
            rv[i] = gv[p < N ? p : N - 1];  // in range for every lane (N >= 1); used only for p < N
        }
    } else {
        const uint2 *gt = (const uint2 *)keys + toff;
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int p = base + i * kWave;
            const uint2 t = gt[p < N ? p : N - 1];
            rk[i] = p < N ? t.x : kSentinel;
            rv[i] = __uint_as_float(t.y);
        }
    }
}

constexpr uint32_t kBucketLimit = 40;

// DET: the fixed summation order (stable ranks, no hash pre-sum, every run
// summed by its head); a separate instance, so the default one keeps its
// registers.
template <int BLOCK, int TMAX, class VT, bool DET = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(TMAX <= 2048 && !DET ? 5 : 1))) void k_sort_compress(SortArgs a) {
    constexpr int NW = BLOCK / kWave;
    constexpr int IPT = TMAX / BLOCK;
    constexpr int NB = TMAX >= 4096 ? TMAX : TMAX / 2;  // buckets of the one-pass path
    constexpr int LOG_NB = (NB >= 4096) ? 12 : (NB >= 2048) ? 11 : (NB >= 1024) ? 10 : 9;
    static_assert((1 << LOG_NB) == NB, "NB must be a power of two");
    static_assert(NW >= 4, "digit scan uses the first 256 threads");
    static_assert(TMAX <= 65536, "16-bit slots");
    constexpr int OFF_KA = 0;
    constexpr int OFF_SA = OFF_KA + 4 * TMAX;
    constexpr int OFF_KB = OFF_SA + 2 * TMAX;
    constexpr int OFF_SB = OFF_KB + 4 * TMAX;
    constexpr int OFF_H = OFF_SB + 2 * TMAX;
    constexpr int HWORDS = (NW * 256 > NB) ? NW * 256 : NB;
    constexpr int OFF_END = OFF_H + HWORDS * 4;
    static_assert(OFF_KB + (int)sizeof(VT) * TMAX <= OFF_END, "values must fit the free half");
    static_assert(NB % BLOCK == 0, "bucket scan: whole buckets per thread");
    __shared__ __align__(16) uint8_t smem[OFF_END];
    __shared__ uint32_t s_wsum[NW];
    __shared__ uint32_t s_red[4 * NW];
    __shared__ uint64_t s_scan[NW + 1];

    uint32_t *keyA = (uint32_t *)(smem + OFF_KA);
    uint16_t *slotA = (uint16_t *)(smem + OFF_SA);
    uint32_t *keyB = (uint32_t *)(smem + OFF_KB);
    uint16_t *slotB = (uint16_t *)(smem + OFF_SB);
    uint32_t *hist = (uint32_t *)(smem + OFF_H);
    VT *vl = (VT *)(smem + OFF_KB);

    const uint32_t lane = lane_id();
    const uint32_t w = threadIdx.x / kWave;
    const int cb = a.cb;
    const uint32_t colmask = cb ? ((1u << cb) - 1u) : 0u;

    if (a.nbins && (int64_t)blockIdx.x >= (int64_t)*a.nbins) return;
    const int64_t b = a.bin0 + blockIdx.x;
    const int64_t row0 = a.binrow0[b];
    const int64_t nrows = a.binrow0[b + 1] - row0;
    const int64_t toff = a.binoff[b] - a.slot0;
    const int64_t N64 = a.binoff[b + 1] - a.binoff[b];
    if (N64 > a.T) return;
    int N = (int)N64;
    if (N > TMAX) {
        if (threadIdx.x == 0) atomic_or_agent(a.err, (uint32_t)kErrTile);
        return;
    }
    if (N == 0) return;
    int64_t base, bend;  // the bin's first entry of C and one past its last
    int32_t *colidx = a.colidx;
    void *cvals = a.cvals;
    int64_t capacity = a.capacity;
    if (a.outs) {
        const OutDesc od = a.outs[prob_of_row(a.prob_row0, a.nprob, row0)];
        base = od.rowptr[row0 - od.row0];
        bend = od.rowptr[row0 + nrows - od.row0];
        colidx = od.colidx;
        cvals = od.val;
        capacity = od.capacity;
    } else {
        base = a.rowptr[row0 - a.row_base];
        bend = a.rowptr[row0 + nrows - a.row_base];
    }
    // padding slots (sentinel keys) are left out of the sort; they are
    // counted so that the sorted tuples occupy [0, Nr)
    uint32_t rk[IPT];
    VT rv[IPT];
    uint32_t kmin = 0xffffffffu, kmax = 0, nreal = 0;
    load_bin<BLOCK, TMAX, VT>(a.keys, a.vals, toff, N, rk, rv);
    // Bins whose keys repeat (at most half of the slots hold
    // distinct keys; that count is known from C's row pointers): equal keys
    // are first summed in an LDS hash table, in double, and only the
    // distinct keys, each with its sum, go on to the sort.
    {
        const int64_t D = bend - base;
        if (!DET && D > 0 && 2 * D <= N && D <= TMAX / 2) {
            constexpr int TSD = TMAX;  // table slots, load factor <= 1/2
            constexpr int LOG_TSD = (TSD >= 4096) ? 12 : (TSD >= 2048) ? 11 : (TSD >= 1024) ? 10 : 9;
            static_assert((1 << LOG_TSD) == TSD, "table size");
            static_assert(TSD % BLOCK == 0, "whole slots per thread");
            uint32_t *tk = (uint32_t *)(smem + OFF_KA);  // table keys
            double *tv = (double *)(smem + OFF_KB);      // table sums
            static_assert(OFF_KA + 4 * TSD <= OFF_KB && OFF_KB + 8 * TSD <= OFF_END, "table fits");
            for (int x = threadIdx.x; x < TSD; x += BLOCK) {
                tk[x] = kSentinel;
                tv[x] = 0.0;
            }
            __syncthreads();
            bool full = false;
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
                if (p < N && rk[i] != kSentinel) {
                    uint32_t h = (rk[i] * 0x9E3779B1u) >> (32 - LOG_TSD);
                    int probes = 0;
                    while (probes < TSD) {
                        const uint32_t old = atomicCAS(&tk[h], kSentinel, rk[i]);
                        if (old == kSentinel || old == rk[i]) break;
                        h = (h + 1) & (TSD - 1);
                        ++probes;
                    }
                    if (probes < TSD) atomicAdd(&tv[h], (double)rv[i]);
                    else full = true;  // more distinct keys than the row pointers say
                }
            }
            if (full) atomic_or_agent(a.err, (uint32_t)kErrTile);
            __syncthreads();
            // compact the occupied slots to the front of the table, in
            // place: every thread holds its slots in registers across the
            // scan's barriers before any is overwritten
            constexpr int SPT = TSD / BLOCK;
            uint32_t ck[SPT];
            double cs[SPT];
            uint32_t occ = 0;
#pragma unroll
            for (int x = 0; x < SPT; ++x) {
                ck[x] = tk[threadIdx.x * SPT + x];
                cs[x] = tv[threadIdx.x * SPT + x];
                occ += ck[x] != kSentinel;
            }
            uint64_t tot;
            uint64_t at = block_excl_scan<BLOCK, SumOp>(occ, s_scan, tot);
            __syncthreads();
#pragma unroll
            for (int x = 0; x < SPT; ++x) {
                if (ck[x] != kSentinel) {
                    tk[at] = ck[x];
                    tv[at] = cs[x];
                    ++at;
                }
            }
            __syncthreads();
            N = (int)tot;
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
                rk[i] = p < N ? tk[p] : kSentinel;
                rv[i] = p < N ? (VT)tv[p] : (VT)0;
            }
            __syncthreads();  // the sort below reuses the LDS
        }
    }
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const bool real = rk[i] != kSentinel;
        if (real) {
            kmin = rk[i] < kmin ? rk[i] : kmin;
            kmax = rk[i] > kmax ? rk[i] : kmax;
        }
        nreal += popc64(ballot(real));
    }
    for (int x = threadIdx.x; x < NB; x += BLOCK) hist[x] = 0;
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        const uint32_t o1 = __shfl_xor(kmin, d, kWave);
        const uint32_t o2 = __shfl_xor(kmax, d, kWave);
        kmin = o1 < kmin ? o1 : kmin;
        kmax = o2 > kmax ? o2 : kmax;
    }
    if (lane == 0) {
        s_red[w] = kmin;
        s_red[NW + w] = kmax;
        s_red[3 * NW + w] = nreal;
    }
    __syncthreads();
    kmin = 0xffffffffu;
    kmax = 0;
    int Nr = 0;
    for (int ww = 0; ww < NW; ++ww) {
        kmin = s_red[ww] < kmin ? s_red[ww] : kmin;
        kmax = s_red[NW + ww] > kmax ? s_red[NW + ww] : kmax;
        Nr += (int)s_red[3 * NW + ww];
    }
    if (Nr == 0) return;  // block-uniform: only padding slots
    const uint32_t span = kmax - kmin;
    const int spanbits = span ? 32 - __clz(span) : 0;
    const int sh = spanbits > LOG_NB ? spanbits - LOG_NB : 0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
        if (rk[i] != kSentinel) atomicAdd(&hist[(rk[i] - kmin) >> sh], 1u);
    }
    __syncthreads();
    {
        constexpr int BPT = NB / BLOCK;
        uint32_t c[BPT];
        uint32_t tsum = 0, tmax = 0;
#pragma unroll
        for (int x = 0; x < BPT; ++x) {
            c[x] = hist[threadIdx.x * BPT + x];
            tsum += c[x];
            tmax = c[x] > tmax ? c[x] : tmax;
        }
        const uint32_t inc = wave_incl_scan_u32(tsum);
#pragma unroll
        for (int d = kWave / 2; d >= 1; d >>= 1) {
            const uint32_t o = __shfl_xor(tmax, d, kWave);
            tmax = o > tmax ? o : tmax;
        }
        if (lane == kWave - 1) s_wsum[w] = inc;
        if (lane == 0) s_red[2 * NW + w] = tmax;
        __syncthreads();
        uint32_t run = inc - tsum;
        for (uint32_t ww = 0; ww < w; ++ww) run += s_wsum[ww];
#pragma unroll
        for (int x = 0; x < BPT; ++x) {
            hist[threadIdx.x * BPT + x] = run;
            run += c[x];
        }
    }
    __syncthreads();
    uint32_t maxbucket = 0;
    for (int ww = 0; ww < NW; ++ww) maxbucket = s_red[2 * NW + ww] > maxbucket ? s_red[2 * NW + ww] : maxbucket;

    if (maxbucket <= kBucketLimit) {
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
            if (rk[i] != kSentinel) {
                const uint32_t pos = atomicAdd(&hist[(rk[i] - kmin) >> sh], 1u);
                keyB[pos] = rk[i];
                slotB[pos] = (uint16_t)p;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int q = (int)w * kWave * IPT + i * kWave + (int)lane;
            if (q < Nr) {
                const uint32_t key = keyB[q];
                const uint32_t bk = (key - kmin) >> sh;
                const uint32_t be = hist[bk];
                const uint32_t bs = bk ? hist[bk - 1] : 0u;
                uint32_t rank = bs;
                if constexpr (!DET) {
                    // equal keys in bucket order (any order sums the same up to rounding)
                    for (uint32_t x = bs; x < be; x += 2) {
                        const uint32_t k0 = keyB[x], k1 = keyB[x + 1];  // x + 1 stays inside the LDS arrays
                        rank += (k0 < key) || (k0 == key && x < (uint32_t)q);
                        if (x + 1 < be) rank += (k1 < key) || (k1 == key && x + 1 < (uint32_t)q);
                    }
                } else {
                    // equal keys in slot order: a stable sort
                    const uint32_t sq = slotB[q];
                    for (uint32_t x = bs; x < be; ++x) {
                        const uint32_t kx = keyB[x];
                        rank += (kx < key) || (kx == key && slotB[x] < sq);
                    }
                }
                keyA[rank] = key;
                slotA[rank] = slotB[q];
            }
        }
        __syncthreads();
    } else {
        // stable LSD radix sort, per-wave ballot ranking
        // row bits cover nrows itself, so a padding slot's sentinel (all ones
        // in the sorted bits) orders after every real key
        const int rowbits = 32 - __clz((uint32_t)nrows);
        const int bits = rowbits + cb;
        const int passes = (bits + 7) / 8;
        const int dw = passes ? (bits + passes - 1) / passes : 0;
        uint32_t *dk = (passes & 1) ? keyA : keyB;
        uint16_t *dsl = (passes & 1) ? slotA : slotB;
        uint32_t *sk = (passes & 1) ? keyB : keyA;
        uint16_t *ssl = (passes & 1) ? slotB : slotA;
        if (passes == 0) {
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
                if (p < N) {
                    keyA[p] = rk[i];
                    slotA[p] = (uint16_t)p;
                }
            }
        }
        uint32_t *wh = hist + w * 256;
        for (int pass = 0; pass < passes; ++pass) {
            const int shift = pass * dw;
            const int width = (bits - shift) < dw ? (bits - shift) : dw;
            const uint32_t R = 1u << width;
            const uint32_t dmask = R - 1;
            __syncthreads();
            for (uint32_t d = lane; d < R; d += kWave) wh[d] = 0;
            uint32_t kv[IPT], sv[IPT], rankdig[IPT];
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
                const bool act = p < N;
                uint32_t key = 0, slot = 0;
                if (act) {
                    key = pass == 0 ? rk[i] : sk[p];
                    slot = pass == 0 ? (uint32_t)p : (uint32_t)ssl[p];
                }
                const uint32_t dig = (key >> shift) & dmask;
                uint64_t peers = ballot(act);
                for (int bt = 0; bt < width; ++bt) {
                    const bool bit = (dig >> bt) & 1u;
                    const uint64_t bb = ballot(act && bit);
                    peers &= bit ? bb : ~bb;
                }
                uint32_t rank = 0;
                if (act) {
                    const uint32_t old = wh[dig];
                    rank = old + popc_lt(peers);
                    if (lane == (uint32_t)__builtin_ctzll(peers)) wh[dig] = old + popc64(peers);
                }
                kv[i] = key;
                sv[i] = slot;
                rankdig[i] = rank | (dig << 16);
            }
            __syncthreads();
            uint32_t tot = 0, inc = 0;
            if (threadIdx.x < 256) {
                if (threadIdx.x < R)
                    for (int ww = 0; ww < NW; ++ww) tot += hist[ww * 256 + threadIdx.x];
                inc = wave_incl_scan_u32(tot);
                if (lane == kWave - 1) s_wsum[w] = inc;
            }
            __syncthreads();
            if (threadIdx.x < R) {
                uint32_t run = inc - tot;
                for (uint32_t ww = 0; ww < w; ++ww) run += s_wsum[ww];
                for (int ww = 0; ww < NW; ++ww) {
                    const uint32_t h = hist[ww * 256 + threadIdx.x];
                    hist[ww * 256 + threadIdx.x] = run;
                    run += h;
                }
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
                if (p < N) {
                    const uint32_t dig = rankdig[i] >> 16;
                    const uint32_t dest = wh[dig] + (rankdig[i] & 0xffffu);
                    dk[dest] = kv[i];
                    dsl[dest] = (uint16_t)sv[i];
                }
            }
            uint32_t *tk = sk;
            sk = dk;
            dk = tk;
            uint16_t *ts = ssl;
            ssl = dsl;
            dsl = ts;
        }
        __syncthreads();
    }
    // park the values by slot, then sum every run of equal keys and write it
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
        if (p < N) vl[p] = rv[i];
    }
    __syncthreads();
    // run heads (first tuple of each key), counted per wave
    uint32_t wrun = 0;
    uint32_t hr[IPT], kc[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
        bool head = false;
        kc[i] = kSentinel;
        if (p < Nr) {
            kc[i] = keyA[p];
            head = (p == 0) || (kc[i] != keyA[p - 1]);
        }
        const uint64_t hm = ballot(head);
        hr[i] = head ? (wrun + popc_lt(hm)) : 0xffffffffu;
        wrun += popc64(hm);
    }
    if (lane == 0) s_wsum[w] = wrun;
    __syncthreads();
    uint32_t wbase = 0, heads = 0;
    for (uint32_t ww = 0; ww < NW; ++ww) {
        if (ww < w) wbase += s_wsum[ww];
        heads += s_wsum[ww];
    }
    VT *cv = (VT *)cvals;
    if (DET || (uint32_t)Nr - heads <= (uint32_t)Nr / 16) {
        // few repeated keys (or the fixed order): each head sums its run
        // itself, left to right.  The
        // LDS reads of all of a thread's heads are issued together.
        uint32_t hk[IPT], hs[IPT], hn[IPT];
        VT hv[IPT];
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
            const int pc = p < Nr ? p : Nr - 1;
            hk[i] = kc[i];
            hs[i] = slotA[pc];
            hn[i] = p + 1 < Nr ? keyA[p + 1] : kSentinel;
        }
#pragma unroll
        for (int i = 0; i < IPT; ++i) hv[i] = vl[hs[i]];
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            if (hr[i] != 0xffffffffu) {
                const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
                const uint32_t key = hk[i];
                Merge<VT> mg;
                mg.start(hv[i]);
                if (hn[i] == key)
                    for (int q = p + 1; q < Nr && keyA[q] == key; ++q) mg.add(vl[slotA[q]]);
                const int64_t out = base + wbase + hr[i];
                if (out < capacity) {
                    const uint32_t vcol =
                        a.vshift ? ((((uint32_t)row0 + (key >> cb)) & a.vmask) << a.vshift) : 0u;
                    colidx[out] = (int32_t)(vcol | (key & colmask));
                    cv[out] = mg.result();
                } else {
                    atomic_or_agent(a.err, (uint32_t)kErrCapacity);
                }
            }
        }
        return;
    }
    // Many repeated keys: segmented reduction in sorted order: thread t takes sorted positions
    // [t*IPT, t*IPT + IPT) and sums them left to right, restarting at every
    // run head; a segmented scan over the threads carries the sum of a run
    // that started in an earlier thread; the last tuple of each run writes it.
    const int p0 = (int)threadIdx.x * IPT;
    uint32_t ks[IPT];
    Merge<VT> inc[IPT];
    uint32_t hmask = 0;
    Merge<VT> acc;
    acc.zero();
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int p = p0 + j;
        ks[j] = 0;
        if (p < Nr) {
            ks[j] = keyA[p];
            const VT v = vl[slotA[p]];
            if (p == 0 || ks[j] != keyA[p - 1]) {
                hmask |= 1u << j;
                acc.start(v);
            } else {
                acc.add(v);
            }
        }
        inc[j] = acc;
    }
    // exclusive segmented scan of the per-thread (has head, sum) pairs
    bool cf = hmask != 0;
    Merge<VT> ca = acc;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const bool uf = __shfl_up((int)cf, (unsigned)d, kWave) != 0;
        const Merge<VT> ua = shfl_up_merge(ca, d);
        if ((int)lane >= d) {
            if (!cf) ca = merge_cat(ua, ca);
            cf = cf || uf;
        }
    }
    // per-wave totals, then the carry into this thread
    __shared__ Merge<VT> s_wacc[NW];
    __shared__ uint32_t s_wflag[NW];
    if (lane == kWave - 1) {
        s_wacc[w] = ca;
        s_wflag[w] = cf;
    }
    bool xf = __shfl_up((int)cf, 1u, kWave) != 0;
    Merge<VT> xa = shfl_up_merge(ca, 1);
    if (lane == 0) {
        xf = false;
        xa.zero();
    }
    const uint32_t nh = (uint32_t)__builtin_popcount(hmask);
    uint64_t htot;
    const uint64_t hbefore = block_excl_scan<BLOCK, SumOp>(nh, s_scan, htot);  // has barriers
    bool wf = false;
    Merge<VT> wa;
    wa.zero();
    for (uint32_t ww = 0; ww < w; ++ww) {
        if (s_wflag[ww]) {
            wa = s_wacc[ww];
            wf = true;
        } else {
            wa = merge_cat(wa, s_wacc[ww]);
        }
    }
    Merge<VT> carry = xf ? xa : merge_cat(wa, xa);
    uint32_t seen = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int p = p0 + j;
        if (p < Nr) {
            if (hmask & (1u << j)) ++seen;
            const bool tail = (p == Nr - 1) || (keyA[p + 1] != ks[j]);
            if (tail) {
                const Merge<VT> tot = seen ? inc[j] : merge_cat(carry, inc[j]);
                const int64_t out = base + (int64_t)hbefore + seen - 1;
                if (out < capacity) {
                    const uint32_t key = ks[j];
                    const uint32_t vcol =
                        a.vshift ? ((((uint32_t)row0 + (key >> cb)) & a.vmask) << a.vshift) : 0u;
                    colidx[out] = (int32_t)(vcol | (key & colmask));
                    cv[out] = tot.result();
                } else {
                    atomic_or_agent(a.err, (uint32_t)kErrCapacity);
                }
            }
        }
    }
    (void)wf;
}

// Streaming copy with 16-byte accesses, one element per thread
// (bandwidth reference).
__global__ __launch_bounds__(256) void k_copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

}  // namespace pb
