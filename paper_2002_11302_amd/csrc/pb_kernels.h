// PB-SpGEMM kernels for gfx950 (wave64).  No MFMA: nothing here is a dense
// contraction.  Every phase streams HBM; the per-bin sort runs in LDS.
#pragma once
#include "pb_device.h"

namespace pb {

// ---------------------------------------------------------------------------
// Facts the symbolic step leaves on the device (read back once).
struct SymInfo {
    uint64_t flop;       // Algorithm 3's multiplication count
    uint64_t nbins;      // bins of consecutive rows
    uint64_t maxnormal;  // largest row flop among rows <= tile/2
    uint64_t maxrow;     // largest row flop
    uint64_t noversize;  // rows with more tuples than the tile
    uint32_t err;
    uint32_t pad;
};

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// ---------------------------------------------------------------------------
// Single-pass chained scan (decoupled look-back).  Tiles are claimed in
// ticket order; thread t of a tile owns IPT consecutive elements.
// Src(i) -> element payload; Dst(i, exclusive, element) stores results;
// Dst::total(t) receives the grand total (called by the owner of the last
// element); Dst::side(i, e) -> value max-reduced per tile and handed to
// Dst::side_commit.
template <int BLOCK, int IPT, class Op, class Src, class Dst>
__global__ __launch_bounds__(BLOCK) void k_chained_scan(int64_t n, Src src, Dst dst, uint64_t *status,
                                                        uint32_t *ticket, uint32_t *err) {
    constexpr int NW = BLOCK / kWave;
    __shared__ uint64_t s_tmp[NW + 2];
    __shared__ uint64_t s_side[NW];
    __shared__ int64_t s_tile;
    if (threadIdx.x == 0) s_tile = atomic_add_agent(ticket, 1u);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t base = tile * (int64_t)(BLOCK * IPT) + (int64_t)threadIdx.x * IPT;
    uint64_t e[IPT];
    uint64_t local = Op::identity();
    uint64_t side = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t i = base + j;
        e[j] = i < n ? src(i) : Op::identity();
        if (i < n) {
            uint64_t sv = dst.side(i, e[j]);
            side = sv > side ? sv : side;
        }
        local = Op::combine(local, e[j]);
    }
    // tile max of the side values
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        uint64_t o = __shfl_xor(side, d, kWave);
        side = o > side ? o : side;
    }
    if (lane_id() == 0) s_side[threadIdx.x / kWave] = side;
    uint64_t tile_total;
    const uint64_t texcl = block_excl_scan<BLOCK, Op>(local, s_tmp, tile_total);
    if (threadIdx.x == 0) {
        uint64_t mx = 0;
        for (int i = 0; i < NW; ++i) mx = s_side[i] > mx ? s_side[i] : mx;
        dst.side_commit(mx);
        s_tmp[NW + 1] = look_back<Op>(status, tile, tile_total, err);
    }
    __syncthreads();
    uint64_t run = Op::combine(s_tmp[NW + 1], texcl);
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

// Algorithm 3: flop_k = nnz(A(:,k)) * nnz(B(k,:)); F = exclusive scan.
struct ColFlopSrc {
    const int64_t *acp, *brp;
    __device__ uint64_t operator()(int64_t k) const {
        return (uint64_t)((acp[k + 1] - acp[k]) * (brp[k + 1] - brp[k]));
    }
};
struct ColFlopDst : NoSide {
    int64_t *F;
    int64_t K;
    SymInfo *info;
    __device__ void operator()(int64_t k, uint64_t excl, uint64_t) const { F[k] = (int64_t)excl; }
    __device__ void total(uint64_t t) const {
        F[K] = (int64_t)t;
        info->flop = t;
    }
};

// Per-row flop: rowflop[r] = sum over k with A(r,k) stored of nnz(B(k,:)).
// One thread per column of A; columns longer than 32 entries are taken by
// the whole wave, lanes striding over the column.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_rowflop(int64_t K, const int64_t *acp, const int32_t *ari,
                                                   const int64_t *brp, uint64_t *rowflop) {
    const int64_t k = blockIdx.x * (int64_t)BLOCK + threadIdx.x;
    int64_t a0 = 0, na = 0, nb = 0;
    if (k < K) {
        a0 = acp[k];
        na = acp[k + 1] - a0;
        nb = brp[k + 1] - brp[k];
        if (nb == 0) na = 0;
    }
    const bool longcol = na > 32;
    if (!longcol) {
        for (int64_t e = a0; e < a0 + na; ++e) atomic_add_agent(&rowflop[ari[e]], (uint64_t)nb);
    }
    uint64_t mask = ballot(longcol);
    const uint32_t lane = lane_id();
    while (mask) {
        const int L = __builtin_ctzll(mask);
        mask &= mask - 1;
        const int64_t la0 = __shfl(a0, L, kWave);
        const int64_t lna = __shfl(na, L, kWave);
        const int64_t lnb = __shfl(nb, L, kWave);
        for (int64_t e = la0 + lane; e < la0 + lna; e += kWave) atomic_add_agent(&rowflop[ari[e]], (uint64_t)lnb);
    }
}

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

// Bin cut.  With H = T - maxnormal and row weight g(r) = R[r] + c*r
// (c = ceil(H / 2^rowbits) >= 1), a row starts a new bin when it is the
// first row, when it or its predecessor is big (row flop > T/2), or when
// floor(g/H) differs from its predecessor's.  A bin of normal rows then
// holds < H + maxnormal <= T tuples and < H/c <= 2^rowbits rows; a big row
// is a bin by itself.  Payload: (count of starts) << 31 | last start row.
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
    __device__ uint64_t operator()(int64_t r) const {
        const uint64_t thalf = T / 2;
        const uint64_t H = T - info->maxnormal;
        const uint64_t cap = rowbits >= 40 ? (1ull << 40) : (1ull << rowbits);
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
        }
        return start ? ((1ull << 31) | (uint64_t)r) : 0;
    }
};
struct BinDst {
    uint64_t *rowinfo;
    int32_t *binrow0;
    int64_t *binoff;
    const uint64_t *R;
    int64_t m;
    uint64_t T;
    SymInfo *info;
    __device__ void operator()(int64_t r, uint64_t excl, uint64_t e) const {
        const uint64_t incl = BinOp::combine(excl, e);
        const uint64_t bin = (incl >> 31) - 1;
        const uint64_t l = incl & 0x7fffffffull;
        rowinfo[r] = (bin << 32) | (uint64_t)(r - (int64_t)l);
        if (e) {
            binrow0[bin] = (int32_t)r;
            binoff[bin] = (int64_t)R[r];
            if (R[r + 1] - R[r] > T) atomic_add_agent(&info->noversize, (uint64_t)1);
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
// Expand (Algorithm 2's outer-product loop).  The flop space [0, flop) is
// cut into chunks of C = BLOCK*IPT tuples; tuple t lies in column k of A /
// row k of B with F[k] <= t < F[k+1], and is the product of the i-th entry
// of A(:,k) and the j-th entry of B(k,:), (i, j) = divmod(t - F[k], nnz(B(k,:))).
// The tuples from one A entry form a run bound for one bin (its row's);
// the run's first tuple in the chunk reserves room for the whole run piece
// with one atomic on the bin cursor, so each run lands contiguously and
// consecutive lanes write consecutive addresses (the GPU counterpart of the
// paper's cache-line-sized local bins, Section 3.3).
struct ExpandArgs {
    int64_t flop, K;
    const int64_t *F;
    const int32_t *kstart;
    const int64_t *acp;
    const int32_t *ari;
    const double *av;
    const int64_t *brp;
    const int32_t *bci;
    const double *bv;
    const uint64_t *rowinfo;
    const int64_t *binoff;
    uint32_t *bincur;
    uint32_t *keys;
    void *vals;
    int cb;
    uint32_t *err;
};

template <int BLOCK, int IPT, int WMAX, class VT>
__global__ __launch_bounds__(BLOCK) void k_expand(ExpandArgs a) {
    constexpr int C = BLOCK * IPT;
    __shared__ int64_t s_F[WMAX];
    __shared__ uint32_t s_base[C];
    const int64_t c = blockIdx.x;
    const int64_t t0 = c * (int64_t)C;
    const int64_t t1 = (t0 + C < a.flop) ? t0 + C : a.flop;
    const int64_t k0 = a.kstart[c];
    const int64_t kl = a.kstart[c + 1];
    const int64_t nwin = kl - k0 + 2;  // F[k0 .. kl+1]
    const bool windowed = nwin <= WMAX;
    if (windowed)
        for (int64_t i = threadIdx.x; i < nwin; i += BLOCK) s_F[i] = a.F[k0 + i];
    __syncthreads();

    uint32_t r_bin[IPT], r_lpos[IPT], r_key[IPT];
    VT r_val[IPT];
    VT *vals = (VT *)a.vals;
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const int64_t t = t0 + it * BLOCK + threadIdx.x;
        if (t < t1) {
            int64_t k, Fk;
            if (windowed) {
                const int64_t j = last_le(s_F, 0, nwin - 1, t);
                k = k0 + j;
                Fk = s_F[j];
            } else {
                k = last_le(a.F, k0, kl + 1, t);
                Fk = a.F[k];
            }
            const int64_t off = t - Fk;
            const int64_t bs = a.brp[k];
            const int64_t nb = a.brp[k + 1] - bs;
            int64_t i, j;
            if (off < 0x100000000ll && nb < 0x100000000ll) {
                const uint32_t q = (uint32_t)off / (uint32_t)nb;
                i = q;
                j = off - (int64_t)q * nb;
            } else {
                i = off / nb;
                j = off - i * nb;
            }
            const int64_t e = a.acp[k] + i;
            const int32_t r = a.ari[e];
            const uint64_t info = a.rowinfo[r];
            const uint32_t bin = (uint32_t)(info >> 32);
            const uint32_t rl = (uint32_t)info;
            const int64_t q = bs + j;
            const uint32_t col = (uint32_t)a.bci[q];
            const double prod = a.av[e] * a.bv[q];
            const int64_t lstart = (t - j > t0) ? t - j : t0;
            if (j == 0 || t == t0) {
                const int64_t rest = nb - j;
                const int64_t len = (rest < t1 - t) ? rest : t1 - t;
                s_base[t - t0] = atomic_add_agent(&a.bincur[bin], (uint32_t)len);
            }
            r_bin[it] = bin;
            r_lpos[it] = (uint32_t)(lstart - t0);
            r_key[it] = (rl << a.cb) | col;
            r_val[it] = (VT)prod;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
        const int64_t t = t0 + it * BLOCK + threadIdx.x;
        if (t < t1) {
            const uint32_t bin = r_bin[it];
            const int64_t slot = a.binoff[bin] + (int64_t)s_base[r_lpos[it]] + (t - t0 - r_lpos[it]);
            if (slot < a.binoff[bin + 1]) {
                a.keys[slot] = r_key[it];
                vals[slot] = r_val[it];
            } else {
                atomic_or_agent(a.err, (uint32_t)kErrBinOverflow);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Sort + compress + ConvertCSR, one workgroup per bin, bins claimed in row
// order by ticket.  The bin's N <= TMAX tuples are loaded once; keys are
// radix-sorted in LDS (stable LSD, <= 8-bit digits, per-wave ballot ranking)
// together with 16-bit slot numbers; the values stay in registers until the
// keys are sorted and are then parked in LDS by slot.  Equal keys are summed
// in sorted order by the first tuple of each run (Section 3.5's merge), the
// bin's entry count goes through a decoupled look-back over bins to give
// its offset in C, and row pointers of the bin's rows are written from the
// sorted keys (Algorithm 2's ConvertCSR).
struct SortArgs {
    int64_t nbins, m;
    const int32_t *binrow0;
    const int64_t *binoff;
    const uint32_t *keys;
    const void *vals;
    int cb;
    uint64_t *status;
    uint32_t *ticket;
    uint32_t *err;
    int64_t *rowptr;
    int32_t *colidx;
    void *cvals;
    int64_t capacity;
};

template <class VT>
struct Merge;
template <>
struct Merge<double> {
    // plain left-to-right double sum
    double s;
    __device__ void start(double v) { s = v; }
    __device__ void add(double v) { s = s + v; }
    __device__ double result() const { return s; }
};
template <>
struct Merge<float> {
    // Neumaier's compensated sum in float
    float s, c;
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

template <int BLOCK, int TMAX, class VT>
__global__ __launch_bounds__(BLOCK) void k_sort_compress(SortArgs a) {
    constexpr int NW = BLOCK / kWave;
    constexpr int IPT = TMAX / BLOCK;
    static_assert(NW >= 4, "digit scan uses the first 256 threads");
    static_assert(TMAX <= 65536, "16-bit slots");
    constexpr int OFF_KA = 0;
    constexpr int OFF_SA = OFF_KA + 4 * TMAX;
    constexpr int OFF_KB = OFF_SA + 2 * TMAX;
    constexpr int OFF_SB = OFF_KB + 4 * TMAX;
    constexpr int OFF_H = OFF_SB + 2 * TMAX;
    constexpr int OFF_END = OFF_H + NW * 256 * 4;
    static_assert(OFF_KB + (int)sizeof(VT) * TMAX <= OFF_END, "values must fit the free half");
    __shared__ __align__(16) uint8_t smem[OFF_END];
    __shared__ uint32_t s_wsum[NW];
    __shared__ int64_t s_bin, s_base;
    __shared__ uint32_t s_nnzb;

    uint32_t *keyA = (uint32_t *)(smem + OFF_KA);
    uint16_t *slotA = (uint16_t *)(smem + OFF_SA);
    uint32_t *keyB = (uint32_t *)(smem + OFF_KB);
    uint16_t *slotB = (uint16_t *)(smem + OFF_SB);
    uint32_t *hist = (uint32_t *)(smem + OFF_H);
    VT *vl = (VT *)(smem + OFF_KB);

    const uint32_t lane = lane_id();
    const uint32_t w = threadIdx.x / kWave;
    if (threadIdx.x == 0) s_bin = atomic_add_agent(a.ticket, 1u);
    __syncthreads();
    const int64_t b = s_bin;
    const int64_t row0 = a.binrow0[b];
    const int64_t nrows = a.binrow0[b + 1] - row0;
    const int64_t toff = a.binoff[b];
    int N = (int)(a.binoff[b + 1] - toff);
    if (N > TMAX) {
        if (threadIdx.x == 0) atomic_or_agent(a.err, (uint32_t)kErrTile);
        N = 0;
    }
    const int cb = a.cb;
    const VT *gv = (const VT *)a.vals;

    uint32_t rk[IPT];
    VT rv[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
        if (p < N) {
            rk[i] = a.keys[toff + p];
            rv[i] = gv[toff + p];
        }
    }

    const int rowbits = nrows > 1 ? 32 - __clz((uint32_t)(nrows - 1)) : 0;
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
        // digit offsets in (digit, wave) order
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
        __syncthreads();
        uint32_t *tk = sk;
        sk = dk;
        dk = tk;
        uint16_t *ts = ssl;
        ssl = dsl;
        dsl = ts;
    }
    // sorted keys and slots are in keyA / slotA; park values by slot
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
        if (p < N) vl[p] = rv[i];
    }
    __syncthreads();

    // heads of runs of equal keys, ranked in sorted order
    uint32_t hr[IPT];
    uint32_t wrun = 0;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
        bool head = false;
        if (p < N) head = (p == 0) || (keyA[p] != keyA[p - 1]);
        const uint64_t hm = ballot(head);
        hr[i] = head ? (wrun + popc_lt(hm)) : 0xffffffffu;
        wrun += popc64(hm);
    }
    if (lane == 0) s_wsum[w] = wrun;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int ww = 0; ww < NW; ++ww) {
            const uint32_t t = s_wsum[ww];
            s_wsum[ww] = acc;
            acc += t;
        }
        const int64_t base = (int64_t)look_back<SumOp>(a.status, b, (uint64_t)acc, a.err);
        s_base = base;
        if (b == a.nbins - 1) a.rowptr[a.m] = base + acc;
        s_nnzb = acc;
    }
    __syncthreads();
    const int64_t base = s_base;
    const uint32_t nnzb = s_nnzb;
    const uint32_t wbase = s_wsum[w];
    const uint32_t colmask = cb ? ((1u << cb) - 1u) : 0u;
    VT *cv = (VT *)a.cvals;
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int p = (int)w * kWave * IPT + i * kWave + (int)lane;
        if (p < N && hr[i] != 0xffffffffu) {
            const uint32_t key = keyA[p];
            const int64_t out = base + wbase + hr[i];
            Merge<VT> mg;
            mg.start(vl[slotA[p]]);
            for (int q = p + 1; q < N && keyA[q] == key; ++q) mg.add(vl[slotA[q]]);
            if (out < a.capacity) {
                a.colidx[out] = (int32_t)(key & colmask);
                cv[out] = mg.result();
            } else {
                atomic_or_agent(a.err, (uint32_t)kErrCapacity);
            }
            const int64_t rl = cb < 32 ? (int64_t)(key >> cb) : 0;
            const int64_t rlprev = p == 0 ? -1 : (cb < 32 ? (int64_t)(keyA[p - 1] >> cb) : 0);
            for (int64_t rr = rlprev + 1; rr <= rl; ++rr) a.rowptr[row0 + rr] = out;
        }
        if (p == N - 1) {
            const int64_t rl = cb < 32 ? (int64_t)(keyA[p] >> cb) : 0;
            for (int64_t rr = rl + 1; rr < nrows; ++rr) a.rowptr[row0 + rr] = base + nnzb;
        }
    }
    if (N == 0)
        for (int64_t rr = threadIdx.x; rr < nrows; rr += BLOCK) a.rowptr[row0 + rr] = base;
}

// Streaming copy with 16-byte accesses (bandwidth reference).
__global__ __launch_bounds__(256) void k_copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace pb
