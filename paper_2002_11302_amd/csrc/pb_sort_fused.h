// Sort + compress with ConvertCSR fused in (pb_tune.convert = 2).  Same
// sort and merge as k_sort_compress; the difference is where C's row
// pointers come from.  Bins take tickets in launch order; once a bin knows
// how many entries of C it holds (its distinct keys), it publishes that
// count, and a decoupled look-back over the earlier bins' counts gives the
// entries of C before it.  The bin then writes its entries and its rows'
// pointers at their final places, with no count pass and no row scan.
#pragma once
#include "pb_kernels.h"

namespace pb {

constexpr uint64_t kSegStart = 1ull << 61;  // SegSumOp's segment flag

// Fused ConvertCSR, step 1: publish the bin's entry count.  A bin that
// starts a problem of a batch (seg) or the launch (tile 0) needs nothing
// from earlier bins, so it publishes an inclusive prefix right away.
__device__ __forceinline__ void bin_publish(const SortArgs &a, int64_t tile, uint64_t D, bool seg) {
    if (threadIdx.x == 0) {
        const uint64_t agg = (seg ? kSegStart : 0ull) | D;
        atomic_store_agent(&a.status[tile], ((seg || tile == 0) ? kFlagPrefix : kFlagAgg) | agg);
    }
}
// Step 2: the entries of C before the bin (plus those before the launch),
// block-uniform.  Contains a barrier.
__device__ __forceinline__ int64_t bin_resolve(const SortArgs &a, int64_t tile, uint64_t D, bool seg, int64_t *s_base) {
    if (threadIdx.x < kWave) {
        uint64_t ex = 0;
        if (!seg && tile > 0) ex = resolve_prefix_wave<SegSumOp>(a.status, tile, D, a.err) & ~kSegStart;
        if (threadIdx.x == 0) s_base[0] = (int64_t)ex + (a.rowptr_base ? *a.rowptr_base : 0);
    }
    __syncthreads();
    return s_base[0];
}

// Where a bin's results go: its rows' pointers (rp[0] is its first row), C's
// entries, and whether it starts a problem (seg) or ends the launch's rows
// or its problem's (last).
struct BinOut {
    int64_t *rp;
    int32_t *colidx;
    void *cvals;
    int64_t capacity;
    bool seg, last;
};
__device__ __forceinline__ BinOut bin_out(const SortArgs &a, int64_t row0, int64_t nrows) {
    BinOut o;
    if (a.outs) {
        const OutDesc od = a.outs[prob_of_row(a.prob_row0, a.nprob, row0)];
        o.rp = od.rowptr + (row0 - od.row0);
        o.colidx = od.colidx;
        o.cvals = od.val;
        o.capacity = od.capacity;
        o.seg = row0 == od.row0;
        o.last = row0 + nrows == od.row0 + od.m;
    } else {
        o.rp = a.rowptr + (row0 - a.row_base);
        o.colidx = a.colidx;
        o.cvals = a.cvals;
        o.capacity = a.capacity;
        o.seg = false;
        o.last = row0 + nrows == a.rows_end;
    }
    return o;
}

// Fused ConvertCSR for a bin that sorts nothing (no real tuples, or a wide
// row whose D entries were counted elsewhere): all its rows start at the
// entries before it.  Contains a barrier.
__device__ __forceinline__ void bin_without_sort(const SortArgs &a, int64_t tile, int64_t row0, int nrows, uint64_t D,
                                                 int block, int64_t *s_base) {
    const BinOut o = bin_out(a, row0, nrows);
    bin_publish(a, tile, D, o.seg);
    const int64_t base = bin_resolve(a, tile, D, o.seg, s_base);
    for (int y = threadIdx.x; y < nrows; y += block) o.rp[y] = base;
    if (o.last && threadIdx.x == 0) o.rp[nrows] = base + (int64_t)D;
}

constexpr int kHashProbeLimit = 64;  // fused: an insert probing further abandons the hash path

// Sums equal keys of the bin in an LDS hash table (in double) and leaves
// only the distinct keys, each with its sum, in rk / rv (the first N after
// the call).  Returns the number of distinct keys, or -1 (rk / rv untouched)
// when an insert probes more than `plimit` slots or more than half of the
// table would be needed.  Uses the first 14 * TMAX bytes of smem.  Contains
// barriers: call from every thread.
template <int BLOCK, int TMAX, class VT>
__device__ __forceinline__ int hash_sum(uint32_t (&rk)[TMAX / BLOCK], VT (&rv)[TMAX / BLOCK], int &N, int plimit,
                                        uint8_t *smem, uint32_t *s_red, uint64_t *s_scan) {
    constexpr int NW = BLOCK / kWave;
    constexpr int IPT = TMAX / BLOCK;
    constexpr int TSD = TMAX;  // table slots
    constexpr int LOG_TSD = (TSD >= 4096) ? 12 : (TSD >= 2048) ? 11 : (TSD >= 1024) ? 10 : 9;
    static_assert((1 << LOG_TSD) == TSD, "table size");
    static_assert(TSD % BLOCK == 0, "whole slots per thread");
    const uint32_t lane = lane_id();
    const uint32_t w = threadIdx.x / kWave;
    uint32_t *tk = (uint32_t *)smem;             // table keys
    double *tv = (double *)(smem + 6 * TMAX);    // table sums
    for (int x = threadIdx.x; x < TSD; x += BLOCK) {
        tk[x] = kSentinel;
        tv[x] = 0.0;
    }
    __syncthreads();
    uint32_t fresh = 0, failed = 0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
        if (p < N && rk[i] != kSentinel) {
            uint32_t h = (rk[i] * 0x9E3779B1u) >> (32 - LOG_TSD);
            int probes = 0;
            uint32_t old = 0;
            while (probes < plimit) {
                old = atomicCAS(&tk[h], kSentinel, rk[i]);
                if (old == kSentinel || old == rk[i]) break;
                h = (h + 1) & (TSD - 1);
                ++probes;
            }
            if (probes < plimit) {
                atomicAdd(&tv[h], (double)rv[i]);
                fresh += old == kSentinel;
            } else {
                failed = 1;
            }
        }
    }
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        fresh += __shfl_xor(fresh, d, kWave);
        failed |= __shfl_xor(failed, d, kWave);
    }
    if (lane == 0) {
        s_red[w] = fresh;
        s_red[NW + w] = failed;
    }
    __syncthreads();
    uint32_t D = 0, anyfail = 0;
    for (int ww = 0; ww < NW; ++ww) {
        D += s_red[ww];
        anyfail |= s_red[NW + ww];
    }
    __syncthreads();
    if (anyfail || 2 * D > (uint32_t)TMAX) return -1;
    // compact the occupied slots to the front of the table, in place: every
    // thread holds its slots in registers across the scan's barriers before
    // any is overwritten
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
    __syncthreads();  // the sort reuses the LDS
    return (int)D;
}


template <int BLOCK, int TMAX, class VT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(TMAX <= 2048 ? 5 : 1))) void k_sort_compress_fused(
    SortArgs a) {
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
    __shared__ int64_t s_x[2];  // [0] the bin's ticket, [1] entries of C before the bin

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
    if (threadIdx.x == 0) s_x[0] = (int64_t)atomic_add_agent(a.ticket, 1u);
    __syncthreads();
    const int64_t tile = s_x[0];
    const int64_t b = a.bin0 + tile;
    const int64_t row0 = a.binrow0[b];
    const int nrows = (int)(a.binrow0[b + 1] - row0);  // at most the tile
    const int64_t N64 = a.binoff[b + 1] - a.binoff[b];
    // bins with nothing to sort here: a wide row (counted elsewhere), no
    // tuples, or (an internal error) more tuples than the tile
    if (N64 > a.T || N64 == 0 || N64 > TMAX) {
        if (N64 <= a.T && N64 > TMAX && threadIdx.x == 0) atomic_or_agent(a.err, (uint32_t)kErrTile);
        const uint64_t D = N64 > a.T ? (uint64_t)a.bignnz[row0 - a.row_base] : 0ull;
        bin_without_sort(a, tile, row0, nrows, D, BLOCK, &s_x[1]);
        return;
    }
    int N = (int)N64;
    bool published = false;
    // padding slots (sentinel keys) are left out of the sort; they are
    // counted so that the sorted tuples occupy [0, Nr)
    uint32_t rk[IPT];
    VT rv[IPT];
    load_bin<BLOCK, TMAX, VT>(a.keys, a.vals, a.binoff[b] - a.slot0, N, rk, rv);
    uint32_t kmin, kmax, maxbucket;
    int Nr, sh;
    kmin = 0xffffffffu;
    kmax = 0;
    uint32_t nreal = 0;
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
    Nr = 0;
    for (int ww = 0; ww < NW; ++ww) {
        kmin = s_red[ww] < kmin ? s_red[ww] : kmin;
        kmax = s_red[NW + ww] > kmax ? s_red[NW + ww] : kmax;
        Nr += (int)s_red[3 * NW + ww];
    }
    if (Nr == 0) {  // block-uniform: only padding slots
        bin_without_sort(a, tile, row0, nrows, 0, BLOCK, &s_x[1]);
        return;
    }
    const uint32_t span = kmax - kmin;
    const int spanbits = span ? 32 - __clz(span) : 0;
    sh = spanbits > LOG_NB ? spanbits - LOG_NB : 0;
#pragma unroll
    for (int i = 0; i < IPT; ++i)
        if (rk[i] != kSentinel) atomicAdd(&hist[(rk[i] - kmin) >> sh], 1u);
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
    maxbucket = 0;
    for (int ww = 0; ww < NW; ++ww) maxbucket = s_red[2 * NW + ww] > maxbucket ? s_red[2 * NW + ww] : maxbucket;
    bool bucketed = maxbucket <= kBucketLimit;
    if (!bucketed) {
        // crowded buckets: first try summing repeated keys; the distinct
        // keys (if they fit the table) go to the radix sort
        const int Dh = hash_sum<BLOCK, TMAX, VT>(rk, rv, N, kHashProbeLimit, smem, s_red, s_scan);
        if (Dh >= 0) {
            bin_publish(a, tile, (uint64_t)Dh, bin_out(a, row0, nrows).seg);
            published = true;
            Nr = Dh;
        }
    }

    if (bucketed) {
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
                for (uint32_t x = bs; x < be; x += 2) {
                    const uint32_t k0 = keyB[x], k1 = keyB[x + 1];  // x + 1 stays inside the LDS arrays
                    rank += (k0 < key) || (k0 == key && x < (uint32_t)q);
                    if (x + 1 < be) rank += (k1 < key) || (k1 == key && x + 1 < (uint32_t)q);
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
    uint32_t hr[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
        bool head = false;
        if (p < Nr) head = (p == 0) || (keyA[p] != keyA[p - 1]);
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
    const BinOut o = bin_out(a, row0, nrows);
    int64_t *const rp = o.rp;
    // the bin's entries of C are its distinct keys
    if (!published) bin_publish(a, tile, heads, o.seg);
    const int64_t base = bin_resolve(a, tile, heads, o.seg, &s_x[1]);  // the bin's first entry of C
    {
        // rows after the row of the bin's last key
        const int lastrow = (int)(cb < 32 ? (keyA[Nr - 1] >> cb) : 0u);
        for (int y = lastrow + 1 + threadIdx.x; y < nrows; y += BLOCK) rp[y] = base + heads;
        if (o.last && threadIdx.x == 0) rp[nrows] = base + heads;
    }
    int32_t *const colidx = o.colidx;
    VT *const cv = (VT *)o.cvals;
    const int64_t capacity = o.capacity;
    if ((uint32_t)Nr - heads <= (uint32_t)Nr / 16) {
        // few repeated keys: each head sums its (short) run itself.  The
        // LDS reads of all of a thread's heads are issued together.
        uint32_t hk[IPT], hs[IPT], hn[IPT];
        VT hv[IPT];
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
            const int pc = p < Nr ? p : Nr - 1;
            hk[i] = keyA[pc];
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
                {
                    // the first entry of its row starts the rows since the
                    // previous entry's row
                    const int row = (int)(cb < 32 ? (key >> cb) : 0u);
                    const int prow = p == 0 ? -1 : (int)(cb < 32 ? (keyA[p - 1] >> cb) : 0u);
                    for (int y = prow + 1; y <= row; ++y) rp[y] = out;
                }
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
    Merge<VT> wa;
    wa.zero();
    for (uint32_t ww = 0; ww < w; ++ww) {
        if (s_wflag[ww]) wa = s_wacc[ww];
        else wa = merge_cat(wa, s_wacc[ww]);
    }
    Merge<VT> carry = xf ? xa : merge_cat(wa, xa);
    uint32_t seen = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int p = p0 + j;
        if (p < Nr) {
            if (hmask & (1u << j)) {
                ++seen;
                {
                    const int row = (int)(cb < 32 ? (ks[j] >> cb) : 0u);
                    const uint32_t pk = j ? ks[j - 1] : (p ? keyA[p - 1] : 0u);
                    const int prow = p == 0 ? -1 : (int)(cb < 32 ? (pk >> cb) : 0u);
                    const int64_t ob = base + (int64_t)hbefore + seen - 1;
                    for (int y = prow + 1; y <= row; ++y) rp[y] = ob;
                }
            }
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
}


}  // namespace pb
