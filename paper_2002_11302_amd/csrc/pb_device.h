// Device helpers shared by the PB-SpGEMM kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pb {

constexpr int kWave = 64;

// Device-side error bits, OR-ed into a status word in the workspace.
enum : uint32_t {
    kErrSpin = 1u,      // a look-back wait of the fused ConvertCSR gave up (should never happen)
    kErrBinOverflow = 2u,  // an expand append ran past its bin (inconsistent inputs)
    kErrCapacity = 4u,  // C had less room than nnz(C)
    kErrTile = 8u,      // a bin larger than the sort tile reached the sort kernel
    kErrWide = 16u,     // a wide row's column window exceeds the tile and the dense accumulator
    kErrGrid = 32u,     // more bins than the launch bound (internal)
};

// Upper bound on look-back polls before a wait is abandoned with kErrSpin;
// at ~64 cycles per poll this is well under a second.
constexpr uint32_t kSpinCap = 1u << 24;

// Key of a padding slot (no tuple).  No real key reaches it: the bin cut
// keeps the row part of every key below its all-ones value.
constexpr uint32_t kSentinel = 0xffffffffu;

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
// number of set bits of m below this lane
__device__ __forceinline__ uint32_t popc_lt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__builtin_popcountll(m); }

template <class T>
__device__ __forceinline__ T atomic_add_agent(T *p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T atomic_load_agent(T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ void atomic_store_agent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T atomic_max_agent(T *p, T v) {
    return __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T atomic_or_agent(T *p, T v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Look-back status word: [63:62] flag, [61:0] payload.
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagPrefix = 2ull << 62;
constexpr uint64_t kPayload = (1ull << 62) - 1;

// Sum of non-negative counts (< 2^62).
struct SumOp {
    static __device__ __forceinline__ uint64_t identity() { return 0; }
    static __device__ __forceinline__ uint64_t combine(uint64_t a, uint64_t b) { return a + b; }
};

template <class Op>
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t o = __shfl_up(v, (unsigned)d, kWave);
        if (lane >= (uint32_t)d) v = Op::combine(o, v);
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint32_t o = __shfl_up(v, (unsigned)d, kWave);
        if (lane >= (uint32_t)d) v += o;
    }
    return v;
}

// Exclusive scan over the block of one value per thread.  `lds` needs
// BLOCK/64 + 1 words.  Returns the exclusive prefix; `total` receives the
// block total.  Contains barriers: call from every thread.
template <int BLOCK, class Op>
__device__ uint64_t block_excl_scan(uint64_t v, uint64_t *lds, uint64_t &total) {
    constexpr int NW = BLOCK / kWave;
    const uint32_t lane = lane_id();
    const uint32_t w = threadIdx.x / kWave;
    uint64_t incl = wave_incl_scan<Op>(v);
    if (lane == kWave - 1) lds[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t acc = Op::identity();
        for (int i = 0; i < NW; ++i) {
            uint64_t t = lds[i];
            lds[i] = acc;
            acc = Op::combine(acc, t);
        }
        lds[NW] = acc;
    }
    __syncthreads();
    uint64_t excl = __shfl_up(incl, 1u, kWave);
    if (lane == 0) excl = Op::identity();
    uint64_t r = Op::combine(lds[w], excl);
    total = lds[NW];
    __syncthreads();
    return r;
}

// Decoupled look-back, wave-wide.  Tiles (workgroups) are numbered in the
// order they started (a ticket), and each publishes in status[tile] first
// its aggregate (kFlagAgg), then its inclusive prefix (kFlagPrefix).
// resolve_prefix_wave, called by one whole wave (all 64 lanes active) of a
// tile that has published its aggregate `agg`, polls 64 predecessors per
// round trip (lane l reads tile p - l), stops at the nearest inclusive
// prefix, combines the payloads in between in tile order, publishes the
// tile's inclusive prefix and returns its exclusive prefix in every lane
// (identity for tile 0, which publishes its prefix directly).  Predecessor
// tiles belong to workgroups that started earlier and never wait on later
// tiles, so every wait ends; the spin cap only guards against corrupted
// status words.
template <class Op>
__device__ uint64_t resolve_prefix_wave(uint64_t *status, int64_t tile, uint64_t agg, uint32_t *err) {
    const uint32_t lane = lane_id();
    if (tile == 0) return Op::identity();
    uint64_t acc = Op::identity();  // combination of the tiles passed so far
    int64_t p = tile - 1;
    uint32_t spins = 0;
    while (true) {
        const int64_t idx = p - (int64_t)lane;
        const uint64_t wv = idx >= 0 ? atomic_load_agent(&status[idx]) : kFlagPrefix;
        const uint64_t flag = wv & ~kPayload;
        const uint64_t pm = ballot(flag == kFlagPrefix);
        const uint64_t zm = ballot(flag == 0);
        const uint32_t f = pm ? (uint32_t)__builtin_ctzll(pm) : 64u;
        const uint64_t need = f >= 63 ? ~0ull : ((2ull << f) - 1);  // lanes 0..f
        if (zm & need) {
            if (++spins > kSpinCap) {
                if (lane == 0) atomic_or_agent(err, (uint32_t)kErrSpin);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        // combine lanes f..0 (tile order: higher lane = earlier tile)
        uint64_t v = lane <= f ? (wv & kPayload) : Op::identity();
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint64_t o = __shfl_down(v, (unsigned)d, kWave);
            if (lane + d < (uint32_t)kWave) v = Op::combine(o, v);
        }
        v = __shfl(v, 0, kWave);
        acc = Op::combine(v, acc);
        if (f < 64) break;
        p -= kWave;
    }
    if (lane == 0) atomic_store_agent(&status[tile], kFlagPrefix | Op::combine(acc, agg));
    return acc;
}

// largest i in [lo, hi) with a[i] <= x, given a[lo] <= x (a non-decreasing)
template <class T>
__device__ __forceinline__ int64_t last_le(const T *a, int64_t lo, int64_t hi, T x) {
    while (hi - lo > 1) {
        int64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] <= x) lo = mid;
        else hi = mid;
    }
    return lo;
}

}  // namespace pb
