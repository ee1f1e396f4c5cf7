// Host runtime of the PB-SpGEMM library: C ABI, validation, workspace
// layout, kernel launches.  The contract is in include/pbspgemm.h.
#include "pbspgemm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pb_big.h"
#include "pb_kernels.h"
#include "pb_sort_fused.h"

using namespace pb;

namespace {

thread_local std::string g_last_error;

pb_status fail(pb_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define PB_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) return fail(PB_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define PB_LAUNCHED(name)                                                             \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess) return fail(PB_ERR_HIP, "launch %s: %s", name, hipGetErrorString(e_)); \
    } while (0)

#define PB_TRY(expr)                \
    do {                            \
        pb_status s_ = (expr);      \
        if (s_ != PB_OK) return s_; \
    } while (0)

// Kernel shapes.
constexpr int kScanBlock = 256, kScanIpt = 8, kScanTile = kScanBlock * kScanIpt;
constexpr int64_t kScanDirect = 1024;  // tiles up to which k_scan_apply sums the earlier totals itself
constexpr int kSortBlock = 512, kSortTmax = 4096;
constexpr int kSortBlockSmall = 256, kSortTmaxSmall = 2048;
constexpr int kCountBlock = 512, kCountBlockSmall = 256;
// Default tiles: 2048-tuple bins for a single product (the small sort kernel
// keeps five workgroups per CU); 4096 for a batch, whose rows must each fit
// one bin.
constexpr int kDefaultTile = 2048, kDefaultTileBatched = 4096;
constexpr int kDefaultChunk = 1024;

constexpr int64_t kMaxDim = (1ll << 31) - 1;
constexpr int64_t kMaxCount = (1ll << 62) - 1;

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Carves aligned sub-buffers out of one workspace (or only sizes them).
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base((char *)b) {}
    template <class T>
    T *take(int64_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += (size_t)(count > 0 ? count : 0) * sizeof(T);
        return p;
    }
    size_t mark() const { return (off + 255) & ~(size_t)255; }
};

// ---- profiling -----------------------------------------------------------
struct ProfRec {
    int phase;
    hipEvent_t e0, e1;
};
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<ProfRec> recs;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};
Profiler g_prof;

struct ProfScope {
    hipStream_t st;
    int phase;
    hipEvent_t e0 = nullptr;
    ProfScope(hipStream_t s, int ph) : st(s), phase(ph) {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        if (!g_prof.on) return;
        e0 = g_prof.get();
        if (e0 && hipEventRecord(e0, st) != hipSuccess) e0 = nullptr;
    }
    ~ProfScope() {
        if (!e0) return;
        std::lock_guard<std::mutex> lk(g_prof.mu);
        hipEvent_t e1 = g_prof.get();
        if (!e1) return;
        if (hipEventRecord(e1, st) != hipSuccess) return;
        g_prof.recs.push_back({phase, e0, e1});
    }
};

pb_status check_csx(const pb_csx *x, const char *name) {
    if (!x) return fail(PB_ERR_ARG, "%s is NULL", name);
    if (x->nrows < 0 || x->ncols < 0 || x->nnz < 0) return fail(PB_ERR_SHAPE, "%s has a negative size", name);
    if (x->nrows > kMaxDim || x->ncols > kMaxDim) return fail(PB_ERR_RANGE, "%s dimension exceeds 2^31-1", name);
    if (x->nnz > kMaxCount) return fail(PB_ERR_RANGE, "%s nnz exceeds 2^62", name);
    if (!x->ptr) return fail(PB_ERR_ARG, "%s.ptr is NULL", name);
    if (x->nnz > 0 && (!x->idx || !x->val)) return fail(PB_ERR_ARG, "%s.idx/val is NULL with nnz > 0", name);
    return PB_OK;
}

// Content check of an operand, on when PB_VALIDATE=1 is in the environment
// (a debugging aid; the kernels otherwise trust the inputs): ptr[0] = 0,
// ptr non-decreasing, ptr[major] = nnz, every index in [0, minor) and
// strictly increasing inside its line.  The arrays are copied to the host
// (stream-ordered), so no kernel ever runs on an operand that fails.
bool validate_enabled() {
    const char *v = getenv("PB_VALIDATE");
    return v && v[0] == '1';
}

pb_status validate_csx(const pb_csx *x, const char *name, bool csc, hipStream_t st) {
    const int64_t major = csc ? x->ncols : x->nrows, minor = csc ? x->nrows : x->ncols;
    std::vector<int64_t> ptr((size_t)major + 1);
    std::vector<int32_t> idx((size_t)x->nnz);
    PB_HIP(hipMemcpyAsync(ptr.data(), x->ptr, sizeof(int64_t) * ptr.size(), hipMemcpyDeviceToHost, st));
    if (x->nnz) PB_HIP(hipMemcpyAsync(idx.data(), x->idx, sizeof(int32_t) * idx.size(), hipMemcpyDeviceToHost, st));
    PB_HIP(hipStreamSynchronize(st));
    const char *line = csc ? "column" : "row";
    if (ptr[0] != 0) return fail(PB_ERR_ARG, "%s: ptr[0] is %lld, not 0", name, (long long)ptr[0]);
    if (ptr[(size_t)major] != x->nnz)
        return fail(PB_ERR_ARG, "%s: ptr[%lld] is %lld, not nnz = %lld", name, (long long)major,
                    (long long)ptr[(size_t)major], (long long)x->nnz);
    for (int64_t j = 0; j < major; ++j) {
        const int64_t s = ptr[(size_t)j], e = ptr[(size_t)j + 1];
        if (e < s) return fail(PB_ERR_ARG, "%s: ptr decreases at %s %lld", name, line, (long long)j);
        if (e > x->nnz) return fail(PB_ERR_ARG, "%s: ptr exceeds nnz at %s %lld", name, line, (long long)j);
        for (int64_t q = s; q < e; ++q) {
            const int32_t v = idx[(size_t)q];
            if (v < 0 || v >= minor)
                return fail(PB_ERR_ARG, "%s: index %d out of [0, %lld) in %s %lld", name, v, (long long)minor, line,
                            (long long)j);
            if (q > s && v <= idx[(size_t)q - 1])
                return fail(PB_ERR_ARG, "%s: indices not strictly increasing in %s %lld", name, line, (long long)j);
        }
    }
    return PB_OK;
}

int col_bits(int64_t n) {
    if (n <= 1) return 0;
    return 64 - __builtin_clzll((uint64_t)(n - 1));
}

// PB_TUNE in the environment ("key=value" pairs separated by ',' or ';',
// keys named as the pb_tune fields) fills the fields the caller left at 0.
pb_status apply_env_tune(pb_tune *t) {
    const char *env = getenv("PB_TUNE");
    if (!env || !*env) return PB_OK;
    std::string spec(env);
    size_t pos = 0;
    while (pos <= spec.size()) {
        size_t end = spec.find_first_of(",;", pos);
        if (end == std::string::npos) end = spec.size();
        std::string item = spec.substr(pos, end - pos);
        pos = end + 1;
        const size_t a = item.find_first_not_of(" \t"), z = item.find_last_not_of(" \t");
        if (a == std::string::npos) continue;
        item = item.substr(a, z - a + 1);
        const size_t eq = item.find('=');
        if (eq == std::string::npos) return fail(PB_ERR_ARG, "PB_TUNE: '%s' is not key=value", item.c_str());
        auto trim = [](std::string x) {
            const size_t b = x.find_first_not_of(" \t"), e = x.find_last_not_of(" \t");
            return b == std::string::npos ? std::string() : x.substr(b, e - b + 1);
        };
        const std::string key = trim(item.substr(0, eq)), val = trim(item.substr(eq + 1));
        char *stop = nullptr;
        const long long v = strtoll(val.c_str(), &stop, 10);
        if (val.empty() || !stop || *stop) return fail(PB_ERR_ARG, "PB_TUNE: '%s' is not an integer", val.c_str());
        auto fill32 = [&](int32_t &f) -> pb_status {
            if (v < INT32_MIN || v > INT32_MAX) return fail(PB_ERR_ARG, "PB_TUNE: %s out of range", key.c_str());
            if (f == 0) f = (int32_t)v;
            return PB_OK;
        };
        if (key == "tile_tuples") PB_TRY(fill32(t->tile_tuples));
        else if (key == "expand_chunk") PB_TRY(fill32(t->expand_chunk));
        else if (key == "run_align") PB_TRY(fill32(t->run_align));
        else if (key == "row_count") PB_TRY(fill32(t->row_count));
        else if (key == "convert") PB_TRY(fill32(t->convert));
        else if (key == "deterministic") PB_TRY(fill32(t->deterministic));
        else if (key == "round_tuples") {
            if (t->round_tuples == 0) t->round_tuples = (int64_t)v;
        } else {
            return fail(PB_ERR_ARG, "PB_TUNE: unknown key '%s'", key.c_str());
        }
    }
    return PB_OK;
}

pb_status resolve_tune(const pb_tune *user, int default_tile, int *T, int *chunk, int64_t *round_tuples, int *align,
                       int *rowcount, int *convert, int *det) {
    *T = default_tile;
    *chunk = kDefaultChunk;
    *round_tuples = 0;
    *align = 0;
    *rowcount = 0;
    *convert = 1;
    *det = 0;
    pb_tune eff{};
    if (user) eff = *user;
    PB_TRY(apply_env_tune(&eff));
    const pb_tune *t = &eff;
    if (t->deterministic != 0 && t->deterministic != 1) return fail(PB_ERR_ARG, "deterministic must be 0 or 1");
    *det = t->deterministic;
    if (*det && t->convert == 2) return fail(PB_ERR_ARG, "deterministic mode takes convert 0 or 1");
    if (*det && t->row_count == 1) return fail(PB_ERR_ARG, "deterministic mode needs row buckets (row_count 0 or 2)");
    if (t->convert < 0 || t->convert > 2) return fail(PB_ERR_ARG, "convert must be 0 (auto), 1 or 2");
    *convert = t->convert ? t->convert : 1;
    if (t->row_count < 0 || t->row_count > 2) return fail(PB_ERR_ARG, "row_count must be 0 (auto), 1 or 2");
    *rowcount = t->row_count;
    if (t->run_align != 0 && t->run_align != 1 && t->run_align != 4 && t->run_align != 8)
        return fail(PB_ERR_ARG, "run_align must be 0 (auto), 1, 4 or 8");
    *align = t->run_align;
    if (t->round_tuples < 0) return fail(PB_ERR_ARG, "round_tuples must be >= 0");
    *round_tuples = t->round_tuples;
    if (t->tile_tuples) {
        if (t->tile_tuples < 256 || t->tile_tuples > kSortTmax)
            return fail(PB_ERR_ARG, "tile_tuples must be in [256, %d]", kSortTmax);
        *T = t->tile_tuples;
    }
    if (t->expand_chunk) {
        if (t->expand_chunk != 256 && t->expand_chunk != 512 && t->expand_chunk != 1024 && t->expand_chunk != 2048)
            return fail(PB_ERR_ARG, "expand_chunk must be 256, 512, 1024 or 2048");
        *chunk = t->expand_chunk;
    }
    return PB_OK;
}

}  // namespace

// ---- plan ----------------------------------------------------------------
struct pb_plan {
    // the (block-diagonal, for a batch) product: C is m x n, inner dimension k
    int64_t m = 0, k = 0, n = 0, nnzA = 0, nnzB = 0;
    int32_t count = 1;  // problems in the device tables (1 for a single product)
    int64_t round_tuples = 0;  // requested tuple budget per round (0: no limit)
    int32_t user_count = 1;
    pb_precision prec = PB_F64;
    int T = kDefaultTile, chunk = kDefaultChunk, cb = 0;
    int align = 1;  // run alignment in tuple slots
    int rowcount = 1;  // per-row flop: 1 device atomics, 2 row buckets
    int convert = 1;   // ConvertCSR: 1 count pass + row scan, 2 fused into the sort
    int det = 0;       // fixed summation order (runs in column order of A, stable sort, left-to-right sums)
    // symbolic workspace tables
    SymInfo *info = nullptr;
    int64_t *F = nullptr;
    uint64_t *R = nullptr;
    RowTab *rowtab = nullptr;
    uint64_t *ent = nullptr;  // per A entry: run destination (ent_pack)
    int32_t *binrow0 = nullptr;
    int64_t *binoff = nullptr;
    // batch: packed inputs and problem tables (in the symbolic workspace)
    ProbDesc *pdesc = nullptr;
    int64_t *prob_row0 = nullptr;
    int64_t *acp = nullptr, *brp = nullptr;
    int32_t *ari = nullptr, *bci = nullptr;
    double *av = nullptr, *bv = nullptr;
    std::vector<ProbDesc> hdesc;     // host copy (shapes and bases)
    std::vector<int64_t> prob_flop;  // per-problem multiplications
    void *pinned = nullptr;          // host staging for descriptor uploads
    size_t pinned_bytes = 0;
    hipEvent_t staged = nullptr;     // recorded after a batched call's uploads from the staging area
    bool staged_pending = false;
    // host facts
    SymInfo h{};
    int64_t nchunks = 0;
    size_t ws_bytes = 0;
    // rounds and wide rows (single products whose tuples exceed the round
    // budget, or that have rows wider than the tile)
    bool rounds_mode = false;
    int wbits = 0, lognwin = 0;
    int64_t Tv = 0;  // tile of the virtual rows of wide rows (bins, and the dense accumulator above it)
    struct Round {
        int64_t r0 = 0, r1 = 0, b0 = 0, b1 = 0;  // rows and bins of the round
        int64_t slot0 = 0, flop = 0;              // first slot (R[r0]) and tuples
        int64_t nbig = 0, bigflop = 0, nchunks = 0, nvirt = 0, nvbins = 0, ndense = 0;
        size_t stage_off = 0, stage_bytes = 0;    // wide-row tables in the pinned staging area
        size_t ws_bytes = 0;
    };
    std::vector<Round> rounds;
    ~pb_plan() {
        if (staged) (void)hipEventDestroy(staged);
        if (pinned) (void)hipHostFree(pinned);
    }
};

namespace {

struct SymLayout {
    SymInfo *info;
    uint64_t *stF, *stR, *stB;  // scan tile totals
    uint64_t *R;
    int64_t *F;
    RowTab *rowtab;
    uint32_t *runpos;  // device atomics only: each entry's run offset in its row
    uint64_t *ent;
    int32_t *binrow0;
    int64_t *binoff;
    // row buckets (rowcount 2)
    uint64_t *stH;
    int32_t *kstart;
    uint32_t *hist;
    uint64_t *gflop;
    uint32_t *rec, *roff;
    uint32_t *posof;
    uint64_t *entrec;
    uint32_t *recent, *lste, *lsts, *lstp;  // fixed order only
    int nbkt, ngrp;
    int64_t epw, cpw;
    // batch only
    ProbDesc *pdesc;
    int64_t *prob_row0;
    int64_t *acp, *brp;
    int32_t *ari, *bci;
    double *av, *bv;
    size_t zero_bytes, total;
};

// Shape of the row-bucket distribution: buckets of kRowBucketRows rows;
// workgroups over ranges of kBucketEntries entries of A (the histogram then
// has at most nnz(A) * m / 2^25 <= nnz(A) counts).
constexpr int64_t kBucketEntries = 8192;
struct BucketShape {
    int nbkt, ngrp;
    int64_t epw, cpw;
    int64_t nhist() const { return (int64_t)nbkt * ngrp; }
};
BucketShape bucket_shape(int64_t m, int64_t k, int64_t nnza) {
    BucketShape s{};
    s.nbkt = (int)ceil_div(m, kRowBucketRows);
    s.epw = kBucketEntries;
    s.ngrp = (int)ceil_div(nnza, s.epw);
    s.cpw = s.ngrp ? ceil_div(k, (int64_t)s.ngrp) : 0;
    return s;
}

// Row buckets when A has fewer than 2^32 entries (32-bit positions) and the
// bucket histogram fits LDS; device atomics otherwise.
int pick_rowcount(int requested, int64_t m, int64_t k, int64_t nnza) {
    const bool ok = m > 0 && k > 0 && nnza > 0 && nnza < ((int64_t)1 << 32) &&
                    ceil_div(m, kRowBucketRows) <= kMaxRowBuckets;
    if (requested == 1) return 1;
    if (requested == 2) return ok ? 2 : -1;
    return ok ? 2 : 1;
}

SymLayout sym_layout(void *base, int64_t m, int64_t k, int64_t nnza, int64_t nnzb, int32_t count, int rowcount,
                     int det) {
    Carver cv(base);
    SymLayout L{};
    BucketShape bs{};
    if (rowcount == 2) bs = bucket_shape(m, k, nnza);
    L.nbkt = bs.nbkt;
    L.ngrp = bs.ngrp;
    L.epw = bs.epw;
    L.cpw = bs.cpw;
    // zeroed region first
    L.info = cv.take<SymInfo>(1);
    L.stF = cv.take<uint64_t>(ceil_div(k, kScanTile) + 1);
    L.stR = cv.take<uint64_t>(ceil_div(m, kScanTile) + 1);
    L.stB = cv.take<uint64_t>(ceil_div(m, kScanTile) + 1);
    L.R = cv.take<uint64_t>(m + 1);
    L.stH = rowcount == 2 ? cv.take<uint64_t>(ceil_div(bs.nhist(), kScanTile) + 1) : nullptr;
    L.zero_bytes = cv.mark();
    L.F = cv.take<int64_t>(k + 1);
    L.rowtab = cv.take<RowTab>(m);
    L.runpos = cv.take<uint32_t>(rowcount == 2 ? 0 : nnza);
    L.ent = cv.take<uint64_t>(nnza);
    L.binrow0 = cv.take<int32_t>(m + 1);
    L.binoff = cv.take<int64_t>(m + 1);
    if (rowcount == 2) {
        L.kstart = cv.take<int32_t>(bs.ngrp + 1);
        L.hist = cv.take<uint32_t>(bs.nhist() + 1);
        L.gflop = cv.take<uint64_t>(bs.ngrp);
        L.rec = cv.take<uint32_t>(nnza);
        L.roff = cv.take<uint32_t>(nnza);
        L.posof = cv.take<uint32_t>(nnza);
        L.entrec = cv.take<uint64_t>(nnza);
        if (det) {
            L.recent = cv.take<uint32_t>(nnza);
            L.lste = cv.take<uint32_t>(nnza);
            L.lsts = cv.take<uint32_t>(nnza);
            L.lstp = cv.take<uint32_t>(nnza);
        }
    }
    if (count > 1) {
        L.pdesc = cv.take<ProbDesc>(count);
        L.prob_row0 = cv.take<int64_t>(count);
        L.acp = cv.take<int64_t>(k + 1);
        L.brp = cv.take<int64_t>(k + 1);
        L.ari = cv.take<int32_t>(nnza);
        L.bci = cv.take<int32_t>(nnzb);
        L.av = cv.take<double>(nnza);
        L.bv = cv.take<double>(nnzb);
    }
    L.total = cv.mark();
    return L;
}

struct NumLayout {
    uint32_t *err, *sticket;  // sticket: fused ConvertCSR's bin order
    uint64_t *status, *sstatus;  // row-pointer scan tile totals; fused ConvertCSR's bin status
    int32_t *kstart;
    uint32_t *rownnz;
    OutDesc *outs;
    uint32_t *keys;
    void *vals;
    size_t zero_bytes, total;
};

NumLayout num_layout(void *base, const pb_plan *p) {
    Carver cv(base);
    NumLayout L{};
    L.err = cv.take<uint32_t>(2);
    L.sticket = L.err + 1;
    L.status = cv.take<uint64_t>(ceil_div(p->m, kScanTile) + 1);
    L.sstatus = cv.take<uint64_t>((int64_t)p->h.nbins + 1);
    L.zero_bytes = cv.mark();
    L.kstart = cv.take<int32_t>(p->nchunks + 1);
    L.rownnz = cv.take<uint32_t>(p->m);
    L.outs = p->count > 1 ? cv.take<OutDesc>(p->count) : nullptr;
    const int64_t flop = (int64_t)p->h.slots;
    // tuples (TupleArr): FP64 keys and values apart, FP32c {key, value} words
    if (p->prec == PB_F64) {
        L.keys = cv.take<uint32_t>(flop);
        L.vals = cv.take<double>(flop);
    } else {
        L.keys = (uint32_t *)cv.take<uint2>(flop);
        L.vals = nullptr;
    }
    L.total = cv.mark();
    return L;
}

pb_status fill_zero(void *p, size_t bytes, hipStream_t st) {
    const int64_t n = (int64_t)(bytes / 4);
    if (n <= 0) return PB_OK;
    int64_t grid = ceil_div(n, 256);
    if (grid > 4096) grid = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)grid), dim3(256), 0, st, (uint32_t *)p, n, 0u);
    PB_LAUNCHED("fill");
    return PB_OK;
}

// part: ceil(n / kScanTile) words of scratch for the tile totals.
template <class Op, class Src, class Dst>
pb_status launch_scan(int64_t n, Src src, Dst dst, uint64_t *part, hipStream_t st, const char *name) {
    if (n <= 0) return PB_OK;
    const int64_t tiles = ceil_div(n, kScanTile);
    hipLaunchKernelGGL((k_scan_tiles<kScanBlock, kScanIpt, Op, Src>), dim3((unsigned)tiles), dim3(kScanBlock), 0, st, n,
                       src, part);
    PB_LAUNCHED(name);
    // up to kScanDirect tiles each tile combines the totals before it itself
    const bool prefixed = tiles > kScanDirect;
    if (prefixed) {
        hipLaunchKernelGGL((k_scan_parts<kScanBlock, Op>), dim3(1), dim3(kScanBlock), 0, st, tiles, part);
        PB_LAUNCHED(name);
    }
    hipLaunchKernelGGL((k_scan_apply<kScanBlock, kScanIpt, Op, Src, Dst>), dim3((unsigned)tiles), dim3(kScanBlock), 0,
                       st, n, src, dst, (const uint64_t *)part, prefixed ? 1 : 0);
    PB_LAUNCHED(name);
    return PB_OK;
}

// Row scan (each row's first slot) and bin cut over the per-row slot counts.
pb_status run_row_bins(pb_plan *p, const SymLayout &L, hipStream_t st) {
    const int64_t m = p->m;
    if (m <= 0) return PB_OK;
    PB_TRY(launch_scan<SumOp>(m, RowFlopSrc{L.R}, RowFlopDst{L.R, m, (uint64_t)(p->T / 2), L.info}, L.stR, st,
                              "row scan"));
    PB_TRY(launch_scan<BinOp>(
        m, BinSrc{L.R, L.info, (uint64_t)p->T, 32 - p->cb, p->count > 1 ? L.prob_row0 : nullptr, p->count, -1},
        BinDst{L.rowtab, L.binrow0, L.binoff, L.R, m, (uint64_t)p->T, L.info, nullptr}, L.stB, st, "bin scan"));
    hipLaunchKernelGGL(k_bin_max, dim3((unsigned)std::min<int64_t>(ceil_div(m, 256), 512)), dim3(256), 0, st, L.binoff,
                       m, L.info);
    PB_LAUNCHED("largest bin");
    return PB_OK;
}

// Symbolic kernels on device arrays (the product's, or the packed batch's):
// flop scan, per-row flop with run offsets, row scan, bin cut.
pb_status run_symbolic(pb_plan *p, const SymLayout &L, const int64_t *acp, const int32_t *ari, const int64_t *brp,
                       hipStream_t st) {
    const int64_t m = p->m, k = p->k;
    if (k > 0) {
        PB_TRY(launch_scan<SumOp>(k, ColFlopSrc{acp, brp, p->align}, ColFlopDst{{}, L.F, k, L.info}, L.stF, st,
                                  "flop scan"));
        if (p->rowcount == 2) {
            RowBucketArgs ra{};
            ra.K = k;
            ra.nnz = p->nnzA;
            ra.acp = acp;
            ra.brp = brp;
            ra.ari = ari;
            ra.align = p->align;
            ra.epw = L.epw;
            ra.nbkt = L.nbkt;
            ra.ngrp = L.ngrp;
            ra.cpw = L.cpw;
            ra.kstart = L.kstart;
            ra.hist = L.hist;
            ra.gflop = L.gflop;
            ra.rec = L.rec;
            ra.roff = L.roff;
            ra.posof = L.posof;
            ra.rowflop = L.R;
            ra.info = L.info;
            ra.rowtab = L.rowtab;
            ra.entrec = L.entrec;
            ra.ent = L.ent;
            ra.recent = L.recent;
            ra.lste = L.lste;
            ra.lsts = L.lsts;
            ra.lstp = L.lstp;
            ra.det_tmax = p->T;
            const int64_t nh = (int64_t)L.nbkt * L.ngrp;
            const size_t lds = (size_t)L.nbkt * sizeof(uint32_t);
            const dim3 grid((unsigned)L.ngrp), block(kBucketBlock);
            hipLaunchKernelGGL(k_bucket_hist<kBucketBlock>, grid, block, lds, st, ra);
            PB_LAUNCHED("bucket histogram");
            PB_TRY(launch_scan<SumOp>(nh, HistSrc{L.hist}, HistDst{{}, L.hist, nh}, L.stH, st,
                                      "bucket scan"));
            hipLaunchKernelGGL(k_bucket_scatter<kBucketBlock>, grid, block, lds, st, ra);
            PB_LAUNCHED("bucket scatter");
            if (p->det) hipLaunchKernelGGL(k_bucket_count_det<512>, dim3((unsigned)L.nbkt), dim3(512), 0, st, ra, m);
            else hipLaunchKernelGGL(k_bucket_count<512>, dim3((unsigned)L.nbkt), dim3(512), 0, st, ra, m);
            PB_LAUNCHED("bucket count");
            PB_TRY(run_row_bins(p, L, st));
            if (p->det) hipLaunchKernelGGL(k_bucket_dest_rows<256>, dim3((unsigned)L.nbkt, 8), dim3(256), 0, st, ra, m);
            else hipLaunchKernelGGL(k_bucket_dest<1024>, dim3((unsigned)L.nbkt), dim3(1024), 0, st, ra, m);
            PB_LAUNCHED("bucket destinations");
            hipLaunchKernelGGL(k_bucket_offsets<kBucketBlock>, grid, block, 0, st, ra);
            PB_LAUNCHED("bucket offsets");
        } else {
            hipLaunchKernelGGL(k_rowflop<256>, dim3((unsigned)ceil_div(k, 256)), dim3(256), 0, st, k, acp, ari, brp,
                               p->align, L.R, L.runpos, L.info);
            PB_LAUNCHED("rowflop");
            PB_TRY(run_row_bins(p, L, st));
            if (p->nnzA > 0) {
                hipLaunchKernelGGL(k_entry_dest, dim3((unsigned)ceil_div(p->nnzA, 256)), dim3(256), 0, st, p->nnzA,
                                   ari, L.runpos, L.rowtab, L.ent);
                PB_LAUNCHED("entry destinations");
            }
        }
    } else {
        PB_TRY(fill_zero(L.F, sizeof(int64_t), st));
        PB_TRY(run_row_bins(p, L, st));
    }
    return PB_OK;
}

// Sort + compress launch for `nbins` bins of at most T tuples (T picks the
// kernel shape).
#define PB_SORT_LAUNCH(KERNEL)                                                                                   \
    do {                                                                                                         \
        if (T <= kSortTmaxSmall) {                                                                               \
            if (f64)                                                                                             \
                hipLaunchKernelGGL((KERNEL<kSortBlockSmall, kSortTmaxSmall, double>), dim3((unsigned)nbins),     \
                                   dim3(kSortBlockSmall), 0, st, sa);                                            \
            else                                                                                                 \
                hipLaunchKernelGGL((KERNEL<kSortBlockSmall, kSortTmaxSmall, float>), dim3((unsigned)nbins),      \
                                   dim3(kSortBlockSmall), 0, st, sa);                                            \
        } else {                                                                                                 \
            if (f64)                                                                                             \
                hipLaunchKernelGGL((KERNEL<kSortBlock, kSortTmax, double>), dim3((unsigned)nbins), dim3(kSortBlock), \
                                   0, st, sa);                                                                   \
            else                                                                                                 \
                hipLaunchKernelGGL((KERNEL<kSortBlock, kSortTmax, float>), dim3((unsigned)nbins), dim3(kSortBlock), \
                                   0, st, sa);                                                                   \
        }                                                                                                        \
    } while (0)

// The fixed-order instances of the sort kernel, named for the launch macro.
template <int BLOCK, int TMAX, class VT>
constexpr auto k_sort_compress_det = k_sort_compress<BLOCK, TMAX, VT, true>;

// Sort + compress launch for `nbins` bins of at most T tuples (T picks the
// kernel shape; sa.fused the ConvertCSR mode).
pb_status launch_sort(const pb_plan *p, int64_t T, const SortArgs &sa, int64_t nbins, hipStream_t st) {
    const bool f64 = p->prec == PB_F64;
    if (sa.fused) PB_SORT_LAUNCH(k_sort_compress_fused);
    else if (sa.det) PB_SORT_LAUNCH(k_sort_compress_det);
    else PB_SORT_LAUNCH(k_sort_compress);
    PB_LAUNCHED("sort+compress");
    return PB_OK;
}

// ---- rounds and wide rows ---------------------------------------------------
pb_status ensure_pinned(pb_plan *p, size_t bytes);

// Device layout of one round's numeric workspace.  The zeroed region comes
// first; the wide-row tables (bigs, bige, cpre, bigr) are one block, in the
// order of the pinned staging copy.
struct RoundLayout {
    uint32_t *err;
    uint32_t *sort_ticket;  // fused ConvertCSR: bin order
    SymInfo *rinfo, *vinfo;
    uint64_t *st_rows, *st_cols, *st_v, *st_vb, *st_sort;
    uint32_t *cnt_v, *cur_v;
    size_t zero_bytes;
    int64_t *astart;
    uint64_t *colflop;
    int64_t *F;
    int32_t *kstart;
    uint32_t *rownnz;
    char *bigtab;
    int64_t *bigs, *bige, *cpre;
    int32_t *bigr;
    uint32_t *chist;
    uint64_t *Rv;
    RowTab *vrowtab;
    int32_t *vbinrow0;
    int64_t *vbinoff;
    int32_t *dense;
    uint32_t *rownnz_v;
    int64_t *rowptr_v;
    uint32_t *keys2;
    void *vals2;
    uint32_t *keys;
    void *vals;
    size_t total;
};

size_t big_tables_bytes(int64_t nbig) {
    Carver cv(nullptr);
    cv.take<int64_t>(nbig);
    cv.take<int64_t>(nbig);
    cv.take<int64_t>(nbig + 1);
    cv.take<int32_t>(nbig);
    return cv.mark();
}

RoundLayout round_layout(void *base, const pb_plan *p, const pb_plan::Round &rd) {
    Carver cv(base);
    RoundLayout L{};
    const bool partial = rd.r0 > 0 || rd.r1 < p->m;
    const int64_t nrows = rd.r1 - rd.r0;
    const int vb = p->prec == PB_F64 ? 8 : 4;
    L.err = cv.take<uint32_t>(2);
    L.sort_ticket = L.err + 1;
    L.rinfo = cv.take<SymInfo>(1);
    L.vinfo = cv.take<SymInfo>(1);
    L.st_rows = cv.take<uint64_t>(ceil_div(nrows, kScanTile) + 1);
    L.st_cols = cv.take<uint64_t>(partial ? ceil_div(p->k, kScanTile) + 1 : 0);
    L.st_v = cv.take<uint64_t>(ceil_div(rd.nvirt, kScanTile) + 1);
    L.st_vb = cv.take<uint64_t>(ceil_div(rd.nvirt, kScanTile) + 1);
    L.st_sort = cv.take<uint64_t>(rd.b1 - rd.b0 + 1);
    L.cnt_v = cv.take<uint32_t>(rd.nvirt);
    L.cur_v = cv.take<uint32_t>(rd.nvirt);
    L.zero_bytes = cv.mark();
    L.astart = cv.take<int64_t>(partial ? p->k : 0);
    L.colflop = cv.take<uint64_t>(partial ? p->k : 0);
    L.F = cv.take<int64_t>(partial ? p->k + 1 : 0);
    L.kstart = cv.take<int32_t>(ceil_div(rd.flop, p->chunk) + 1);
    L.rownnz = cv.take<uint32_t>(nrows);
    L.bigtab = cv.take<char>((int64_t)(rd.nbig ? big_tables_bytes(rd.nbig) : 0));
    if (rd.nbig) {
        Carver tc(L.bigtab);
        L.bigs = tc.take<int64_t>(rd.nbig);
        L.bige = tc.take<int64_t>(rd.nbig);
        L.cpre = tc.take<int64_t>(rd.nbig + 1);
        L.bigr = tc.take<int32_t>(rd.nbig);
    }
    L.chist = cv.take<uint32_t>(rd.nchunks << p->lognwin);
    L.Rv = cv.take<uint64_t>(rd.nbig ? rd.nvirt + 1 : 0);
    L.vrowtab = cv.take<RowTab>(rd.nvirt);
    L.vbinrow0 = cv.take<int32_t>(rd.nbig ? rd.nvirt + 1 : 0);
    L.vbinoff = cv.take<int64_t>(rd.nbig ? rd.nvirt + 1 : 0);
    L.dense = cv.take<int32_t>(rd.ndense);
    L.rownnz_v = cv.take<uint32_t>(rd.nvirt);
    L.rowptr_v = cv.take<int64_t>(rd.nbig ? rd.nvirt + 1 : 0);
    // tuples (TupleArr): FP64 keys and values apart, FP32c {key, value} words
    if (vb == 8) {
        L.keys2 = cv.take<uint32_t>(rd.bigflop);
        L.vals2 = cv.take<double>(rd.bigflop);
        L.keys = cv.take<uint32_t>(rd.flop);
        L.vals = cv.take<double>(rd.flop);
    } else {
        L.keys2 = (uint32_t *)cv.take<uint2>(rd.bigflop);
        L.vals2 = nullptr;
        L.keys = (uint32_t *)cv.take<uint2>(rd.flop);
        L.vals = nullptr;
    }
    L.total = cv.mark();
    return L;
}

// Cut the bins into rounds (consecutive bins, at most round_tuples tuples
// each unless one bin alone is larger) and list every round's wide rows.
// Reads the bin tables back once.
// Tile of the virtual rows (a wide row's tuples in one column window).  Their
// bins hold at most this many tuples and are sorted by the small sort kernel,
// and a window with more tuples goes to the dense accumulator.  These windows
// compress well (hub rows), and several smaller workgroups per CU sort them
// faster than 4096-tuple bins, while 2048-tuple windows are still cheaper to
// sort than to accumulate over 4096 columns.  Windows wider than the
// accumulator keep the product's tile (a window above it is unsupported).
constexpr int64_t kVirtualTile = 2048;
int64_t virtual_tile(int64_t T, int wbits) { return wbits <= kDenseBits ? std::min(T, kVirtualTile) : T; }

pb_status build_rounds(pb_plan *p, hipStream_t st) {
    const int64_t nbins = (int64_t)p->h.nbins;
    std::vector<int32_t> brow(nbins + 1);
    std::vector<int64_t> boff(nbins + 1);
    PB_HIP(hipMemcpyAsync(brow.data(), p->binrow0, sizeof(int32_t) * (nbins + 1), hipMemcpyDeviceToHost, st));
    PB_HIP(hipMemcpyAsync(boff.data(), p->binoff, sizeof(int64_t) * (nbins + 1), hipMemcpyDeviceToHost, st));
    PB_HIP(hipStreamSynchronize(st));
    p->rounds_mode = true;
    p->lognwin = std::max(0, std::min(kMaxLogWin, p->cb - kDenseBits));
    p->wbits = p->cb - p->lognwin;
    p->Tv = virtual_tile(p->T, p->wbits);
    const int64_t budget = p->round_tuples > 0 ? p->round_tuples : INT64_MAX;
    const int64_t T = p->T;
    const int64_t vmax = (int64_t)1 << 30;  // virtual rows per round (32-bit bin tables)
    p->rounds.clear();
    int64_t b = 0;
    while (b < nbins) {
        pb_plan::Round rd;
        rd.b0 = b;
        int64_t acc = 0, nb = 0;
        while (b < nbins) {
            const int64_t sz = boff[b + 1] - boff[b];
            const int64_t nbw = nb + (sz > T ? 1 : 0);
            if (b > rd.b0 && (acc + sz > budget || (nbw << p->lognwin) > vmax)) break;
            acc += sz;
            nb = nbw;
            ++b;
        }
        rd.b1 = b;
        rd.r0 = brow[rd.b0];
        rd.r1 = brow[rd.b1];
        rd.slot0 = boff[rd.b0];
        rd.flop = acc;
        rd.nbig = nb;
        p->rounds.push_back(rd);
    }
    if (p->rounds.empty()) {  // no rows: one empty round keeps the code paths uniform
        pb_plan::Round rd;
        p->rounds.push_back(rd);
    }
    // wide-row tables, staged once in pinned memory
    size_t stage = 0;
    for (auto &rd : p->rounds) {
        rd.stage_off = stage;
        rd.stage_bytes = rd.nbig ? big_tables_bytes(rd.nbig) : 0;
        stage += rd.stage_bytes;
    }
    if (stage) PB_TRY(ensure_pinned(p, stage));
    size_t ws = 0;
    for (auto &rd : p->rounds) {
        if (rd.nbig) {
            Carver tc((char *)p->pinned + rd.stage_off);
            int64_t *bigs = tc.take<int64_t>(rd.nbig);
            int64_t *bige = tc.take<int64_t>(rd.nbig);
            int64_t *cpre = tc.take<int64_t>(rd.nbig + 1);
            int32_t *bigr = tc.take<int32_t>(rd.nbig);
            int64_t i = 0;
            cpre[0] = 0;
            for (int64_t bb = rd.b0; bb < rd.b1; ++bb) {
                const int64_t sz = boff[bb + 1] - boff[bb];
                if (sz <= T) continue;
                bigs[i] = boff[bb] - rd.slot0;
                bige[i] = boff[bb + 1] - rd.slot0;
                bigr[i] = brow[bb];
                cpre[i + 1] = cpre[i] + ceil_div(sz, kBigChunk);
                rd.bigflop += sz;
                ++i;
            }
            rd.nchunks = cpre[rd.nbig];
            rd.nvirt = rd.nbig << p->lognwin;
            // virtual bins: every bin but the segment and oversize starts spans at
            // least Tv/2 of weight (tuples + rows); oversize rows have > Tv tuples
            // (floor(weight / H) changes: weight <= tuples + 2 per row, H >= Tv/2;
            // rows over Tv/2 start a bin and make their successor start one)
            const int64_t over = rd.bigflop / (p->Tv + 1) + 1;
            const int64_t bound = (6 * rd.bigflop + 4 * rd.nvirt) / p->Tv + rd.nbig + 4;
            rd.nvbins = std::min(rd.nvirt, bound);
            rd.ndense = std::min(rd.nvirt, over);
        }
        rd.ws_bytes = round_layout(nullptr, p, rd).total;
        ws = std::max(ws, rd.ws_bytes);
    }
    p->ws_bytes = ws;
    return PB_OK;
}

// One round: rows [r0, r1) of C.  rowptr_out is indexed by row - r0 and has
// r1 - r0 + 1 entries; rowptr_base (or null for 0) holds the number of
// entries of C before the round; colidx / cval are indexed by C position.
pb_status run_round(pb_plan *p, const pb_plan::Round &rd, void *ws, const pb_csx *A, const pb_csx *B,
                    int64_t *rowptr_out, const int64_t *rowptr_base, int32_t *colidx, void *cval, int64_t capacity,
                    hipStream_t st) {
    const RoundLayout L = round_layout(ws, p, rd);
    const bool f64 = p->prec == PB_F64;
    const bool partial = rd.r0 > 0 || rd.r1 < p->m;
    const int64_t nrows = rd.r1 - rd.r0;
    const int64_t K = p->k;
    PB_TRY(fill_zero(ws, L.zero_bytes, st));
    if (rd.nbig)
        PB_HIP(hipMemcpyAsync(L.bigtab, (char *)p->pinned + rd.stage_off, rd.stage_bytes, hipMemcpyHostToDevice, st));
    const int64_t *F = p->F;
    const int64_t *astart = nullptr;
    const int64_t nchunks = ceil_div(rd.flop, p->chunk);
    if (rd.flop > 0) {
        ProfScope ps(st, 1);
        if (partial) {
            hipLaunchKernelGGL(k_round_cols, dim3((unsigned)ceil_div(K, 256)), dim3(256), 0, st, K, A->ptr, A->idx,
                               B->ptr, (int32_t)rd.r0, (int32_t)rd.r1, p->align, L.astart, L.colflop);
            PB_LAUNCHED("round columns");
            PB_TRY(launch_scan<SumOp>(K, U64Src{L.colflop}, ColFlopDst{{}, L.F, K, L.rinfo}, L.st_cols, st,
                                      "round flop scan"));
            F = L.F;
            astart = L.astart;
        }
        hipLaunchKernelGGL(k_chunk_start, dim3((unsigned)ceil_div(nchunks + 1, 256)), dim3(256), 0, st, nchunks,
                           (int64_t)p->chunk, K, F, L.kstart);
        PB_LAUNCHED("chunk start");
        ExpandArgs ea{rd.flop, K, F, L.kstart, A->ptr, A->val, B->ptr, B->idx, B->val, p->ent,
                      L.keys, L.vals, p->cb, L.err, astart, rd.slot0, p->align};
        const unsigned grid = (unsigned)ceil_div(nchunks, 4);
        switch (p->chunk) {
            case 256:
                if (f64) hipLaunchKernelGGL((k_expand<256, double>), dim3(grid), dim3(256), 0, st, ea, nchunks);
                else hipLaunchKernelGGL((k_expand<256, float>), dim3(grid), dim3(256), 0, st, ea, nchunks);
                break;
            case 512:
                if (f64) hipLaunchKernelGGL((k_expand<512, double>), dim3(grid), dim3(256), 0, st, ea, nchunks);
                else hipLaunchKernelGGL((k_expand<512, float>), dim3(grid), dim3(256), 0, st, ea, nchunks);
                break;
            case 2048:
                if (f64) hipLaunchKernelGGL((k_expand<2048, double>), dim3(grid), dim3(256), 0, st, ea, nchunks);
                else hipLaunchKernelGGL((k_expand<2048, float>), dim3(grid), dim3(256), 0, st, ea, nchunks);
                break;
            default:
                if (f64) hipLaunchKernelGGL((k_expand<1024, double>), dim3(grid), dim3(256), 0, st, ea, nchunks);
                else hipLaunchKernelGGL((k_expand<1024, float>), dim3(grid), dim3(256), 0, st, ea, nchunks);
                break;
        }
        PB_LAUNCHED("expand");
    }
    const int64_t nb = rd.b1 - rd.b0;
    const int nwin = 1 << p->lognwin;
    const int kstride = f64 ? 1 : 2;  // TupleArr key stride
    BigArgs ba{rd.nbig, p->lognwin, p->wbits, p->cb, L.bigs, L.bige, L.cpre, L.keys, L.vals, kstride, L.chist, L.cnt_v,
               L.cur_v, L.Rv, L.vrowtab, L.keys2, L.vals2, rd.bigflop, L.err};
    if (rd.nbig) {
        ProfScope ps(st, 4);
        hipLaunchKernelGGL(k_big_hist<512>, dim3((unsigned)rd.nchunks), dim3(512), 0, st, ba);
        PB_LAUNCHED("wide-row histogram");
        PB_TRY(launch_scan<SumOp>(rd.nvirt, U32Src{L.cnt_v}, RowFlopDst{L.Rv, rd.nvirt, (uint64_t)(p->Tv / 2), L.vinfo},
                                  L.st_v, st, "virtual row scan"));
        PB_TRY(launch_scan<BinOp>(rd.nvirt,
                                  BinSrc{L.Rv, L.vinfo, (uint64_t)p->Tv, 32 - p->wbits, nullptr, 0, p->lognwin},
                                  BinDst{L.vrowtab, L.vbinrow0, L.vbinoff, L.Rv, rd.nvirt, (uint64_t)p->Tv, L.vinfo,
                                         L.dense},
                                  L.st_vb, st, "virtual bin scan"));
        if (f64) hipLaunchKernelGGL((k_big_scatter<512, double>), dim3((unsigned)rd.nchunks), dim3(512), 0, st, ba);
        else hipLaunchKernelGGL((k_big_scatter<512, float>), dim3((unsigned)rd.nchunks), dim3(512), 0, st, ba);
        PB_LAUNCHED("wide-row scatter");
    }
    DenseArgs da{L.dense, &L.vinfo->noversize, L.Rv, L.keys2, L.vals2, p->wbits, p->lognwin, L.rownnz_v,
                 L.rowptr_v, colidx, cval, capacity, L.err};
    const unsigned dgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(rd.ndense, 2048));
    // With ConvertCSR fused into the sort, the main bins count their own
    // entries; a wide row's count (the sum over its column windows) must be
    // known before the main sort, and its windows' row pointers come from
    // its row pointer after it.
    const bool fused = p->convert != 1;
    {
        ProfScope ps(st, 3);
        if (nb > 0 && !fused) {
            CountArgs ca{p->binrow0, p->binoff, L.keys, kstride, p->cb, L.rownnz, L.err, p->T, rd.b0, rd.slot0, rd.r0,
                         nullptr};
            if (p->T <= kSortTmaxSmall)
                hipLaunchKernelGGL((k_row_nnz<kCountBlockSmall, kSortTmaxSmall>), dim3((unsigned)nb),
                                   dim3(kCountBlockSmall), 0, st, ca);
            else
                hipLaunchKernelGGL((k_row_nnz<kCountBlock, kSortTmax>), dim3((unsigned)nb), dim3(kCountBlock), 0, st,
                                   ca);
            PB_LAUNCHED("row counts");
        }
        if (rd.nbig) {
            CountArgs cv{L.vbinrow0, L.vbinoff, L.keys2, kstride, p->wbits, L.rownnz_v, L.err, p->Tv, 0, 0, 0,
                         &L.vinfo->nbins};
            if (p->Tv <= kSortTmaxSmall)
                hipLaunchKernelGGL((k_row_nnz<kCountBlockSmall, kSortTmaxSmall>), dim3((unsigned)rd.nvbins),
                                   dim3(kCountBlockSmall), 0, st, cv);
            else
                hipLaunchKernelGGL((k_row_nnz<kCountBlock, kSortTmax>), dim3((unsigned)rd.nvbins), dim3(kCountBlock),
                                   0, st, cv);
            PB_LAUNCHED("virtual row counts");
            if (f64) hipLaunchKernelGGL((k_dense<512, double, false>), dim3(dgrid), dim3(512), 0, st, da);
            else hipLaunchKernelGGL((k_dense<512, float, false>), dim3(dgrid), dim3(512), 0, st, da);
            PB_LAUNCHED("dense counts");
            hipLaunchKernelGGL(k_big_rowsum, dim3((unsigned)ceil_div(rd.nbig, 4)), dim3(256), 0, st, rd.nbig,
                               p->lognwin, L.bigr, rd.r0, L.rownnz_v, L.rownnz);
            PB_LAUNCHED("wide-row sums");
        }
        if (!fused && nrows > 0)
            PB_TRY(launch_scan<SumOp>(nrows, RowNnzSrc{L.rownnz}, RowPtrDst{{}, rowptr_out, nrows, rowptr_base},
                                      L.st_rows, st, "row pointer scan"));
    }
    {
        ProfScope ps(st, 2);
        if (nb > 0) {
            SortArgs sa{};
            sa.binrow0 = p->binrow0;
            sa.binoff = p->binoff;
            sa.keys = L.keys;
            sa.vals = L.vals;
            sa.cb = p->cb;
            sa.err = L.err;
            sa.rowptr = rowptr_out;
            sa.colidx = colidx;
            sa.cvals = cval;
            sa.capacity = capacity;
            sa.nprob = 1;
            sa.T = p->T;
            sa.bin0 = rd.b0;
            sa.slot0 = rd.slot0;
            sa.row_base = rd.r0;
            sa.fused = fused ? 1 : 0;
            sa.ticket = L.sort_ticket;
            sa.status = L.st_sort;
            sa.bignnz = L.rownnz;
            sa.rowptr_base = rowptr_base;
            sa.rows_end = rd.r1;
            sa.det = p->det;
            PB_TRY(launch_sort(p, p->T, sa, nb, st));
        }
        if (rd.nbig) {
            hipLaunchKernelGGL(k_big_rowptr, dim3((unsigned)ceil_div(rd.nbig, 4)), dim3(256), 0, st, rd.nbig,
                               p->lognwin, L.bigr, rd.r0, rowptr_out, L.rownnz_v, L.rowptr_v);
            PB_LAUNCHED("virtual row pointers");
            SortArgs sv{};
            sv.binrow0 = L.vbinrow0;
            sv.binoff = L.vbinoff;
            sv.keys = L.keys2;
            sv.vals = L.vals2;
            sv.cb = p->wbits;
            sv.err = L.err;
            sv.rowptr = L.rowptr_v;
            sv.colidx = colidx;
            sv.cvals = cval;
            sv.capacity = capacity;
            sv.nprob = 1;
            sv.T = p->Tv;
            sv.nbins = &L.vinfo->nbins;
            sv.vshift = p->wbits;
            sv.vmask = (uint32_t)(nwin - 1);
            PB_TRY(launch_sort(p, p->Tv, sv, rd.nvbins, st));
            if (f64) hipLaunchKernelGGL((k_dense<512, double, true>), dim3(dgrid), dim3(512), 0, st, da);
            else hipLaunchKernelGGL((k_dense<512, float, true>), dim3(dgrid), dim3(512), 0, st, da);
            PB_LAUNCHED("dense output");
        }
    }
    return PB_OK;
}

pb_status finish_symbolic(pb_plan *p, hipStream_t st) {
    PB_HIP(hipMemcpyAsync(&p->h, p->info, sizeof(SymInfo), hipMemcpyDeviceToHost, st));
    PB_HIP(hipStreamSynchronize(st));
    if (p->h.err) return fail(PB_ERR_INTERNAL, "symbolic device error 0x%x", p->h.err);
    if (p->m == 0) p->h.nbins = 0;
    if (p->h.slots > kEntSlotMask)
        return fail(PB_ERR_UNSUPPORTED, "the product expands to %llu tuple slots; at most 2^40 - 1 are supported",
                    (unsigned long long)p->h.slots);
    if (p->h.maxrow >= ((uint64_t)1 << 32))
        return fail(PB_ERR_UNSUPPORTED, "a row of C expands to %llu tuples; at most 2^32 - 1 are supported",
                    (unsigned long long)p->h.maxrow);
    if (p->h.noversize && p->det)
        return fail(PB_ERR_UNSUPPORTED,
                    "%llu rows expand to more than %d tuples (largest %lld); the fixed summation order needs every "
                    "row within the tile",
                    (unsigned long long)p->h.noversize, p->T, (long long)p->h.maxrow);
    if (p->h.noversize && p->count > 1)
        return fail(PB_ERR_UNSUPPORTED,
                    "%llu rows expand to more than %d tuples (largest %lld); batched products need every row within "
                    "the tile",
                    (unsigned long long)p->h.noversize, p->T, (long long)p->h.maxrow);
    p->nchunks = ceil_div((int64_t)p->h.slots, p->chunk);
    if (p->h.noversize || (p->round_tuples > 0 && (int64_t)p->h.slots > p->round_tuples)) return build_rounds(p, st);
    p->ws_bytes = num_layout(nullptr, p).total;
    return PB_OK;
}

// Numeric kernels: expand, entries per row, row pointers, sort+compress.
// For a single product `C` is its output; for a batch L.outs holds them.
pb_status run_numeric(pb_plan *p, const NumLayout &L, const int64_t *acp, const int32_t *ari, const double *av,
                      const int64_t *brp, const int32_t *bci, const double *bv, const pb_csr_out *C, hipStream_t st) {
    const int64_t flop = (int64_t)p->h.slots;
    const int64_t nbins = (int64_t)p->h.nbins;
    const bool batch = p->count > 1;
    const bool f64 = p->prec == PB_F64;
    if (flop > 0) {
        hipLaunchKernelGGL(k_chunk_start, dim3((unsigned)ceil_div(p->nchunks + 1, 256)), dim3(256), 0, st, p->nchunks,
                           (int64_t)p->chunk, p->k, p->F, L.kstart);
        PB_LAUNCHED("chunk start");
        ExpandArgs ea{flop, p->k, p->F, L.kstart, acp, av, brp, bci, bv, p->ent, L.keys, L.vals, p->cb, L.err,
                      nullptr, 0, p->align};
        ProfScope ps(st, 1);
        const unsigned grid = (unsigned)ceil_div(p->nchunks, 4);
        switch (p->chunk) {
            case 256:
                if (f64) hipLaunchKernelGGL((k_expand<256, double>), dim3(grid), dim3(256), 0, st, ea, p->nchunks);
                else hipLaunchKernelGGL((k_expand<256, float>), dim3(grid), dim3(256), 0, st, ea, p->nchunks);
                break;
            case 512:
                if (f64) hipLaunchKernelGGL((k_expand<512, double>), dim3(grid), dim3(256), 0, st, ea, p->nchunks);
                else hipLaunchKernelGGL((k_expand<512, float>), dim3(grid), dim3(256), 0, st, ea, p->nchunks);
                break;
            case 2048:
                if (f64) hipLaunchKernelGGL((k_expand<2048, double>), dim3(grid), dim3(256), 0, st, ea, p->nchunks);
                else hipLaunchKernelGGL((k_expand<2048, float>), dim3(grid), dim3(256), 0, st, ea, p->nchunks);
                break;
            default:
                if (f64) hipLaunchKernelGGL((k_expand<1024, double>), dim3(grid), dim3(256), 0, st, ea, p->nchunks);
                else hipLaunchKernelGGL((k_expand<1024, float>), dim3(grid), dim3(256), 0, st, ea, p->nchunks);
                break;
        }
        PB_LAUNCHED("expand");
    }
    if (nbins > 0) {
        const bool fused = p->convert != 1;
        if (!fused) {
            ProfScope ps(st, 3);
            CountArgs ca{p->binrow0, p->binoff, L.keys, f64 ? 1 : 2, p->cb, L.rownnz, L.err, p->T, 0, 0, 0, nullptr};
            if (p->T <= kSortTmaxSmall)
                hipLaunchKernelGGL((k_row_nnz<kCountBlockSmall, kSortTmaxSmall>), dim3((unsigned)nbins),
                                   dim3(kCountBlockSmall), 0, st, ca);
            else
                hipLaunchKernelGGL((k_row_nnz<kCountBlock, kSortTmax>), dim3((unsigned)nbins), dim3(kCountBlock), 0, st,
                                   ca);
            PB_LAUNCHED("row counts");
            if (batch) {
                PB_TRY(launch_scan<SegSumOp>(p->m, SegRowNnzSrc{L.rownnz, p->prob_row0, p->count},
                                             SegRowPtrDst{{}, L.outs, p->prob_row0, p->count}, L.status, st,
                                             "row pointer scan"));
            } else {
                PB_TRY(launch_scan<SumOp>(p->m, RowNnzSrc{L.rownnz}, RowPtrDst{{}, C->rowptr, p->m, nullptr}, L.status, st,
                                          "row pointer scan"));
            }
        }
        SortArgs sa{};
        sa.binrow0 = p->binrow0;
        sa.binoff = p->binoff;
        sa.keys = L.keys;
        sa.vals = L.vals;
        sa.cb = p->cb;
        sa.err = L.err;
        if (batch) {
            sa.outs = L.outs;
            sa.prob_row0 = p->prob_row0;
            sa.nprob = p->count;
        } else {
            sa.rowptr = C->rowptr;
            sa.colidx = C->colidx;
            sa.cvals = C->val;
            sa.capacity = C->capacity;
            sa.nprob = 1;
        }
        sa.T = p->T;
        sa.rows_end = p->m;
        sa.fused = fused ? 1 : 0;
        sa.ticket = L.sticket;
        sa.status = L.sstatus;
        sa.det = p->det;
        ProfScope ps(st, 2);
        PB_TRY(launch_sort(p, p->T, sa, nbins, st));
    }
    return PB_OK;
}

// ---- batch helpers --------------------------------------------------------
pb_status check_batch(int32_t count, const pb_csx *A, const pb_csx *B) {
    if (count < 1) return fail(PB_ERR_ARG, "count must be >= 1");
    if (!A || !B) return fail(PB_ERR_ARG, "A/B arrays are NULL");
    for (int32_t i = 0; i < count; ++i) {
        char na[32], nb[32];
        snprintf(na, sizeof na, "A[%d]", i);
        snprintf(nb, sizeof nb, "B[%d]", i);
        PB_TRY(check_csx(&A[i], na));
        PB_TRY(check_csx(&B[i], nb));
        if (A[i].ncols != B[i].nrows)
            return fail(PB_ERR_SHAPE, "problem %d: A.ncols (%lld) != B.nrows (%lld)", i, (long long)A[i].ncols,
                        (long long)B[i].nrows);
    }
    return PB_OK;
}

// Block-diagonal shapes and bases of a batch.
void batch_shapes(int32_t count, const pb_csx *A, const pb_csx *B, std::vector<ProbDesc> &d, int64_t &m, int64_t &k,
                  int64_t &n, int64_t &nnza, int64_t &nnzb) {
    d.resize(count);
    m = k = n = nnza = nnzb = 0;
    for (int32_t i = 0; i < count; ++i) {
        ProbDesc &x = d[i];
        x.aptr = A[i].ptr;
        x.aidx = A[i].idx;
        x.aval = A[i].val;
        x.bptr = B[i].ptr;
        x.bidx = B[i].idx;
        x.bval = B[i].val;
        x.m = A[i].nrows;
        x.k = A[i].ncols;
        x.n = B[i].ncols;
        x.nnza = A[i].nnz;
        x.nnzb = B[i].nnz;
        x.mbase = m;
        x.kbase = k;
        x.abase = nnza;
        x.bbase = nnzb;
        m += x.m;
        k += x.k;
        nnza += x.nnza;
        nnzb += x.nnzb;
        n = x.n > n ? x.n : n;
    }
}

pb_status ensure_pinned(pb_plan *p, size_t bytes) {
    if (p->pinned_bytes >= bytes) return PB_OK;
    if (p->pinned) (void)hipHostFree(p->pinned);
    p->pinned = nullptr;
    p->pinned_bytes = 0;
    PB_HIP(hipHostMalloc(&p->pinned, bytes, hipHostMallocDefault));
    p->pinned_bytes = bytes;
    return PB_OK;
}

// pinned staging layout: [ProbDesc x count][first rows x count][OutDesc x count]
size_t staging_bytes(int32_t count) { return (sizeof(ProbDesc) + sizeof(int64_t) + sizeof(OutDesc)) * (size_t)count; }
ProbDesc *staged_desc(pb_plan *p) { return (ProbDesc *)p->pinned; }
int64_t *staged_row0(pb_plan *p) { return (int64_t *)((char *)p->pinned + sizeof(ProbDesc) * p->count); }
OutDesc *staged_outs(pb_plan *p) {
    return (OutDesc *)((char *)p->pinned + (sizeof(ProbDesc) + sizeof(int64_t)) * p->count);
}

pb_status launch_pack(pb_plan *p, int what, hipStream_t st) {
    int64_t maxlen = 1;
    for (const ProbDesc &d : p->hdesc) {
        const int64_t l = std::max(d.k + 1, std::max(d.nnza, d.nnzb));
        maxlen = l > maxlen ? l : maxlen;
    }
    int64_t gx = ceil_div(maxlen, 256 * 8);
    gx = gx < 1 ? 1 : (gx > 256 ? 256 : gx);
    hipLaunchKernelGGL(k_pack, dim3((unsigned)gx, (unsigned)p->count), dim3(256), 0, st, p->pdesc, p->count, what,
                       p->acp, p->ari, p->av, p->brp, p->bci, p->bv);
    PB_LAUNCHED("pack");
    return PB_OK;
}

}  // namespace

// Status of a finished numeric step from its device error word.
pb_status numeric_status(uint32_t err, int64_t total, int64_t capacity) {
    if (err & kErrWide)
        return fail(PB_ERR_UNSUPPORTED,
                    "a column window of a wide row exceeds the tile and is wider than the dense accumulator "
                    "(n above 2^22 with a heavily clustered row)");
    if (err & ~(uint32_t)kErrCapacity) return fail(PB_ERR_INTERNAL, "numeric device error 0x%x", err);
    if ((err & kErrCapacity) || total > capacity)
        return fail(PB_ERR_CAPACITY, "C needs %lld entries, capacity %lld", (long long)total, (long long)capacity);
    return PB_OK;
}

namespace {

pb_status numeric_impl(pb_plan *p, const pb_csx *A, const pb_csx *B, void *workspace, size_t workspace_bytes,
                       pb_csr_out *C, int64_t *nnzC, void *hip_stream);

// Device scratch of spgemm_numeric_noalloc: the numeric workspace of plans
// that fit it, in a file-scope device array, so that the call allocates
// nothing.  Each GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, not the
// device array: the device address comes from hipGetSymbolAddress, taken
// once per device (with that device current) and kept in g_scratch_ptr.
constexpr size_t kNoAllocScratchBytes = PB_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

pb_status noalloc_scratch(void **out) {
    int dev = -1;
    PB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PB_ERR_UNSUPPORTED, "device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(PB_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PB_OK;
}

}  // namespace

extern "C" {

const char *spgemm_status_string(pb_status s) {
    switch (s) {
        case PB_OK: return "PB_OK";
        case PB_ERR_ARG: return "PB_ERR_ARG";
        case PB_ERR_SHAPE: return "PB_ERR_SHAPE";
        case PB_ERR_RANGE: return "PB_ERR_RANGE";
        case PB_ERR_WORKSPACE: return "PB_ERR_WORKSPACE";
        case PB_ERR_CAPACITY: return "PB_ERR_CAPACITY";
        case PB_ERR_HIP: return "PB_ERR_HIP";
        case PB_ERR_UNSUPPORTED: return "PB_ERR_UNSUPPORTED";
        case PB_ERR_INTERNAL: return "PB_ERR_INTERNAL";
    }
    return "PB_ERR_UNKNOWN";
}

const char *spgemm_last_error(void) { return g_last_error.c_str(); }

pb_status spgemm_symbolic(const pb_csx *A, const pb_csx *B, int32_t prec, const pb_tune *tune, void *sym_ws,
                          size_t *sym_ws_bytes, void *hip_stream, pb_plan **plan, int64_t *flop,
                          size_t *workspace_bytes) {
    g_last_error.clear();
    PB_TRY(check_csx(A, "A"));
    PB_TRY(check_csx(B, "B"));
    if (A->ncols != B->nrows)
        return fail(PB_ERR_SHAPE, "A.ncols (%lld) != B.nrows (%lld)", (long long)A->ncols, (long long)B->nrows);
    if (prec != PB_F64 && prec != PB_F32C) return fail(PB_ERR_ARG, "unknown precision %d", (int)prec);
    if (!sym_ws_bytes) return fail(PB_ERR_ARG, "sym_ws_bytes is NULL");
    int T, chunk, align, rowreq, convert, det;
    int64_t round_tuples;
    PB_TRY(resolve_tune(tune, kDefaultTile, &T, &chunk, &round_tuples, &align, &rowreq, &convert, &det));
    const int64_t m = A->nrows, k = A->ncols, n = B->ncols;
    const int rowcount = pick_rowcount(rowreq, m, k, A->nnz);
    if (rowcount < 0)
        return fail(PB_ERR_ARG, "row_count 2 needs 0 < nnz(A) < 2^32 and at most %d rows", kMaxRowBuckets * kRowBucketRows);
    if (det && rowcount != 2)
        return fail(PB_ERR_ARG, "deterministic mode needs row buckets: 0 < nnz(A) < 2^32 and at most %d rows",
                    kMaxRowBuckets * kRowBucketRows);
    const size_t need = sym_layout(nullptr, m, k, A->nnz, B->nnz, 1, rowcount, det).total;
    if (!sym_ws) {
        *sym_ws_bytes = need;
        return PB_OK;
    }
    if (*sym_ws_bytes < need)
        return fail(PB_ERR_WORKSPACE, "symbolic workspace has %zu bytes, needs %zu", *sym_ws_bytes, need);
    if (!plan || !flop || !workspace_bytes) return fail(PB_ERR_ARG, "plan/flop/workspace_bytes output is NULL");
    if (B->nnz >= (int64_t)1 << 32) return fail(PB_ERR_RANGE, "nnz(B) must be below 2^32 (32-bit in-row run offsets)");
    const int cb = col_bits(n);
    if (cb > 31) return fail(PB_ERR_RANGE, "n too large for packed keys");

    hipStream_t st = (hipStream_t)hip_stream;
    if (validate_enabled()) {
        PB_TRY(validate_csx(A, "A", true, st));
        PB_TRY(validate_csx(B, "B", false, st));
    }
    SymLayout L = sym_layout(sym_ws, m, k, A->nnz, B->nnz, 1, rowcount, det);
    pb_plan *p = new pb_plan();
    p->rowcount = rowcount;
    p->m = m;
    p->k = k;
    p->n = n;
    p->nnzA = A->nnz;
    p->nnzB = B->nnz;
    p->prec = (pb_precision)prec;
    p->T = T;
    p->chunk = chunk;
    p->cb = cb;
    p->round_tuples = round_tuples;
    p->convert = convert;
    p->det = det;
    // FP64 runs padded to 4 slots (whole 32-byte sectors of values) when B's
    // rows are long enough on average for the padding to cost little next to
    // the partial-sector writes it avoids (measured: ER 2^20 d=16 step -3%;
    // 8 slots saves more in the expand but costs more in the sort, and FP32c
    // gains nothing)
    p->align = align ? align : (prec == PB_F64 && k > 0 && B->nnz >= 12 * k ? 4 : 1);
    p->info = L.info;
    p->F = L.F;
    p->R = L.R;
    p->rowtab = L.rowtab;
    p->ent = L.ent;
    p->binrow0 = L.binrow0;
    p->binoff = L.binoff;
    pb_status rs = fill_zero(sym_ws, L.zero_bytes, st);
    if (rs == PB_OK) {
        ProfScope ps(st, 0);
        rs = run_symbolic(p, L, A->ptr, A->idx, B->ptr, st);
    }
    if (rs == PB_OK) rs = finish_symbolic(p, st);
    if (rs != PB_OK) {
        delete p;
        return rs;
    }
    p->prob_flop.assign(1, (int64_t)p->h.flop);
    *plan = p;
    *flop = (int64_t)p->h.flop;
    *workspace_bytes = p->ws_bytes;
    return PB_OK;
}

pb_status spgemm_numeric(pb_plan *p, const pb_csx *A, const pb_csx *B, void *workspace, size_t workspace_bytes,
                         pb_csr_out *C, int64_t *nnzC, void *hip_stream) {
    g_last_error.clear();
    return numeric_impl(p, A, B, workspace, workspace_bytes, C, nnzC, hip_stream);
}

pb_status spgemm_numeric_noalloc(pb_plan *p, const pb_csx *A, const pb_csx *B, pb_csr_out *C, int64_t *nnzC,
                                 void *hip_stream) {
    g_last_error.clear();
    if (!p) return fail(PB_ERR_ARG, "plan is NULL");
    if (p->ws_bytes > kNoAllocScratchBytes)
        return fail(PB_ERR_WORKSPACE,
                    "the plan's numeric workspace (%zu bytes) exceeds the %zu-byte device scratch of "
                    "spgemm_numeric_noalloc; use spgemm_numeric with a workspace",
                    p->ws_bytes, kNoAllocScratchBytes);
    void *ws = nullptr;
    PB_TRY(noalloc_scratch(&ws));
    return numeric_impl(p, A, B, ws, kNoAllocScratchBytes, C, nnzC, hip_stream);
}

}  // extern "C"

namespace {

pb_status numeric_impl(pb_plan *p, const pb_csx *A, const pb_csx *B, void *workspace, size_t workspace_bytes,
                       pb_csr_out *C, int64_t *nnzC, void *hip_stream) {
    if (!p) return fail(PB_ERR_ARG, "plan is NULL");
    if (p->count != 1) return fail(PB_ERR_ARG, "the plan is a batch plan: use spgemm_batched");
    PB_TRY(check_csx(A, "A"));
    PB_TRY(check_csx(B, "B"));
    if (A->nrows != p->m || A->ncols != p->k || B->ncols != p->n || A->nnz != p->nnzA || B->nnz != p->nnzB)
        return fail(PB_ERR_SHAPE, "A/B differ from the matrices given to the symbolic step");
    if (!C || !C->rowptr) return fail(PB_ERR_ARG, "C or C->rowptr is NULL");
    if (C->capacity < 0) return fail(PB_ERR_SHAPE, "negative capacity");
    if (C->capacity > 0 && (!C->colidx || !C->val)) return fail(PB_ERR_ARG, "C->colidx/val is NULL");
    if (p->ws_bytes > 0 && (!workspace || workspace_bytes < p->ws_bytes))
        return fail(PB_ERR_WORKSPACE, "numeric workspace has %zu bytes, needs %zu", workspace_bytes, p->ws_bytes);

    hipStream_t st = (hipStream_t)hip_stream;
    if (p->m == 0) PB_TRY(fill_zero(C->rowptr, sizeof(int64_t), st));
    if (p->rounds_mode) {
        // the rounds share the workspace; each one's error word is read after
        // it, so a sync per round happens only when nnzC is requested
        uint32_t err_all = 0;
        for (size_t i = 0; i < p->rounds.size(); ++i) {
            const pb_plan::Round &rd = p->rounds[i];
            PB_TRY(run_round(p, rd, workspace, A, B, C->rowptr + rd.r0, i ? C->rowptr + rd.r0 : nullptr, C->colidx,
                             C->val, C->capacity, st));
            if (nnzC) {
                uint32_t err = 0;
                PB_HIP(hipMemcpyAsync(&err, round_layout(workspace, p, rd).err, sizeof(uint32_t),
                                      hipMemcpyDeviceToHost, st));
                PB_HIP(hipStreamSynchronize(st));
                err_all |= err;
            }
        }
        if (nnzC) {
            int64_t total = 0;
            PB_HIP(hipMemcpyAsync(&total, C->rowptr + p->m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            PB_HIP(hipStreamSynchronize(st));
            *nnzC = total;
            return numeric_status(err_all, total, C->capacity);
        }
        return PB_OK;
    }
    NumLayout L = num_layout(workspace, p);
    PB_TRY(fill_zero(workspace, L.zero_bytes, st));
    PB_TRY(run_numeric(p, L, A->ptr, A->idx, A->val, B->ptr, B->idx, B->val, C, st));
    if (nnzC) {
        int64_t total = 0;
        uint32_t err = 0;
        PB_HIP(hipMemcpyAsync(&total, C->rowptr + p->m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        PB_HIP(hipMemcpyAsync(&err, L.err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        PB_HIP(hipStreamSynchronize(st));
        *nnzC = total;
        return numeric_status(err, total, C->capacity);
    }
    return PB_OK;
}

}  // namespace

extern "C" {

pb_status spgemm_plan_rounds(const pb_plan *p, int64_t *nrounds, int64_t *row_begin, int64_t *flop_per_round) {
    if (!p || !nrounds) return fail(PB_ERR_ARG, "NULL argument");
    if (p->count != 1) return fail(PB_ERR_ARG, "batch plans have no rounds");
    if (!p->rounds_mode) {
        *nrounds = 1;
        if (row_begin) {
            row_begin[0] = 0;
            row_begin[1] = p->m;
        }
        if (flop_per_round) flop_per_round[0] = (int64_t)p->h.slots;
        return PB_OK;
    }
    *nrounds = (int64_t)p->rounds.size();
    for (size_t i = 0; i < p->rounds.size(); ++i) {
        if (row_begin) row_begin[i] = p->rounds[i].r0;
        if (flop_per_round) flop_per_round[i] = p->rounds[i].flop;
    }
    if (row_begin) row_begin[p->rounds.size()] = p->rounds.empty() ? 0 : p->rounds.back().r1;
    return PB_OK;
}

pb_status spgemm_numeric_round(pb_plan *p, const pb_csx *A, const pb_csx *B, int64_t round, void *workspace,
                               size_t workspace_bytes, pb_csr_out *C, int64_t *nnzC, void *hip_stream) {
    g_last_error.clear();
    if (!p) return fail(PB_ERR_ARG, "plan is NULL");
    if (!p->rounds_mode) {
        if (round != 0) return fail(PB_ERR_ARG, "round %lld out of range (the plan has one round)", (long long)round);
        return spgemm_numeric(p, A, B, workspace, workspace_bytes, C, nnzC, hip_stream);
    }
    if (round < 0 || round >= (int64_t)p->rounds.size())
        return fail(PB_ERR_ARG, "round %lld out of range (the plan has %zu)", (long long)round, p->rounds.size());
    PB_TRY(check_csx(A, "A"));
    PB_TRY(check_csx(B, "B"));
    if (A->nrows != p->m || A->ncols != p->k || B->ncols != p->n || A->nnz != p->nnzA || B->nnz != p->nnzB)
        return fail(PB_ERR_SHAPE, "A/B differ from the matrices given to the symbolic step");
    if (!C || !C->rowptr) return fail(PB_ERR_ARG, "C or C->rowptr is NULL");
    if (C->capacity < 0) return fail(PB_ERR_SHAPE, "negative capacity");
    if (C->capacity > 0 && (!C->colidx || !C->val)) return fail(PB_ERR_ARG, "C->colidx/val is NULL");
    const pb_plan::Round &rd = p->rounds[(size_t)round];
    if (rd.ws_bytes > 0 && (!workspace || workspace_bytes < rd.ws_bytes))
        return fail(PB_ERR_WORKSPACE, "numeric workspace has %zu bytes, needs %zu", workspace_bytes, rd.ws_bytes);
    hipStream_t st = (hipStream_t)hip_stream;
    if (rd.r1 == rd.r0) PB_TRY(fill_zero(C->rowptr, sizeof(int64_t), st));
    PB_TRY(run_round(p, rd, workspace, A, B, C->rowptr, nullptr, C->colidx, C->val, C->capacity, st));
    if (nnzC) {
        int64_t total = 0;
        uint32_t err = 0;
        PB_HIP(hipMemcpyAsync(&total, C->rowptr + (rd.r1 - rd.r0), sizeof(int64_t), hipMemcpyDeviceToHost, st));
        PB_HIP(hipMemcpyAsync(&err, round_layout(workspace, p, rd).err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        PB_HIP(hipStreamSynchronize(st));
        *nnzC = total;
        return numeric_status(err, total, C->capacity);
    }
    return PB_OK;
}

pb_status spgemm_batched_symbolic(int32_t count, const pb_csx *A, const pb_csx *B, int32_t prec,
                                  const pb_tune *tune, void *sym_ws, size_t *sym_ws_bytes, void *hip_stream,
                                  pb_plan **plan, int64_t *flop, size_t *workspace_bytes) {
    g_last_error.clear();
    PB_TRY(check_batch(count, A, B));
    if (prec != PB_F64 && prec != PB_F32C) return fail(PB_ERR_ARG, "unknown precision %d", (int)prec);
    if (!sym_ws_bytes) return fail(PB_ERR_ARG, "sym_ws_bytes is NULL");
    int T, chunk, align, rowreq, convert, det;
    int64_t round_tuples;
    PB_TRY(resolve_tune(tune, kDefaultTileBatched, &T, &chunk, &round_tuples, &align, &rowreq, &convert, &det));
    std::vector<ProbDesc> hd;
    int64_t m, k, n, nnza, nnzb;
    batch_shapes(count, A, B, hd, m, k, n, nnza, nnzb);
    if (m > kMaxDim || k > kMaxDim) return fail(PB_ERR_RANGE, "batch rows / inner dimension exceed 2^31-1 in total");
    // the device tables always hold at least two problems (a batch of one
    // gets an empty second problem) so that the batch code paths apply
    const int32_t cnt = count > 1 ? count : 2;
    const int rowcount = pick_rowcount(rowreq, m, k, nnza);
    if (rowcount < 0)
        return fail(PB_ERR_ARG, "row_count 2 needs 0 < nnz(A) < 2^32 and at most %d rows", kMaxRowBuckets * kRowBucketRows);
    if (det && rowcount != 2)
        return fail(PB_ERR_ARG, "deterministic mode needs row buckets: 0 < nnz(A) < 2^32 and at most %d rows",
                    kMaxRowBuckets * kRowBucketRows);
    const size_t need = sym_layout(nullptr, m, k, nnza, nnzb, cnt, rowcount, det).total;
    if (!sym_ws) {
        *sym_ws_bytes = need;
        return PB_OK;
    }
    if (*sym_ws_bytes < need)
        return fail(PB_ERR_WORKSPACE, "symbolic workspace has %zu bytes, needs %zu", *sym_ws_bytes, need);
    if (!plan || !flop || !workspace_bytes) return fail(PB_ERR_ARG, "plan/flop/workspace_bytes output is NULL");
    if (nnzb >= (int64_t)1 << 32) return fail(PB_ERR_RANGE, "nnz(B) must be below 2^32 (32-bit in-row run offsets)");
    const int cb = col_bits(n);
    if (cb > 31) return fail(PB_ERR_RANGE, "n too large for packed keys");
    if (validate_enabled()) {
        for (int32_t i = 0; i < count; ++i) {
            char na[32], nb[32];
            snprintf(na, sizeof na, "A[%d]", i);
            snprintf(nb, sizeof nb, "B[%d]", i);
            PB_TRY(validate_csx(&A[i], na, true, (hipStream_t)hip_stream));
            PB_TRY(validate_csx(&B[i], nb, false, (hipStream_t)hip_stream));
        }
    }
    if (count == 1) {
        ProbDesc e{};
        e.mbase = hd[0].m;
        e.kbase = hd[0].k;
        e.abase = hd[0].nnza;
        e.bbase = hd[0].nnzb;
        hd.push_back(e);
    }

    hipStream_t st = (hipStream_t)hip_stream;
    SymLayout L = sym_layout(sym_ws, m, k, nnza, nnzb, cnt, rowcount, det);
    pb_plan *p = new pb_plan();
    p->rowcount = rowcount;
    p->m = m;
    p->k = k;
    p->n = n;
    p->nnzA = nnza;
    p->nnzB = nnzb;
    p->count = cnt;
    p->user_count = count;
    p->prec = (pb_precision)prec;
    p->T = T;
    p->chunk = chunk;
    p->cb = cb;
    p->convert = convert;
    p->det = det;
    p->info = L.info;
    p->F = L.F;
    p->R = L.R;
    p->rowtab = L.rowtab;
    p->ent = L.ent;
    p->binrow0 = L.binrow0;
    p->binoff = L.binoff;
    p->pdesc = L.pdesc;
    p->prob_row0 = L.prob_row0;
    p->acp = L.acp;
    p->brp = L.brp;
    p->ari = L.ari;
    p->bci = L.bci;
    p->av = L.av;
    p->bv = L.bv;
    p->hdesc = hd;
    pb_status rs = ensure_pinned(p, staging_bytes(cnt));
    if (rs == PB_OK) {
        std::memcpy(staged_desc(p), hd.data(), sizeof(ProbDesc) * cnt);
        int64_t *pr = staged_row0(p);
        for (int32_t i = 0; i < cnt; ++i) pr[i] = hd[i].mbase;
        if (hipMemcpyAsync(L.pdesc, staged_desc(p), sizeof(ProbDesc) * cnt, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(L.prob_row0, pr, sizeof(int64_t) * cnt, hipMemcpyHostToDevice, st) != hipSuccess)
            rs = fail(PB_ERR_HIP, "descriptor upload failed");
    }
    if (rs == PB_OK) rs = fill_zero(sym_ws, L.zero_bytes, st);
    if (rs == PB_OK) {
        ProfScope ps(st, 0);
        rs = launch_pack(p, 1, st);
        if (rs == PB_OK) rs = run_symbolic(p, L, L.acp, L.ari, L.brp, st);
    }
    if (rs == PB_OK) rs = finish_symbolic(p, st);
    // per-problem flop: the flop scan at the problems' first columns
    std::vector<int64_t> Fb(cnt + 1, 0);
    for (int32_t i = 0; rs == PB_OK && i <= cnt; ++i) {
        const int64_t col = i < cnt ? hd[i].kbase : k;
        if (hipMemcpyAsync(&Fb[i], L.F + col, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess)
            rs = fail(PB_ERR_HIP, "flop readback failed");
    }
    if (rs == PB_OK && hipStreamSynchronize(st) != hipSuccess) rs = fail(PB_ERR_HIP, "flop readback failed");
    if (rs != PB_OK) {
        delete p;
        return rs;
    }
    p->prob_flop.resize(count);
    for (int32_t i = 0; i < count; ++i) {
        p->prob_flop[i] = Fb[i + 1] - Fb[i];
        flop[i] = p->prob_flop[i];
    }
    *plan = p;
    *workspace_bytes = p->ws_bytes;
    return PB_OK;
}

pb_status spgemm_batched(pb_plan *p, int32_t count, const pb_csx *A, const pb_csx *B, void *workspace,
                         size_t workspace_bytes, pb_csr_out *C, int64_t *nnzC, void *hip_stream) {
    g_last_error.clear();
    if (!p) return fail(PB_ERR_ARG, "plan is NULL");
    if (p->count < 2) return fail(PB_ERR_ARG, "the plan is a single-product plan: use spgemm_numeric");
    if (count != p->user_count) return fail(PB_ERR_SHAPE, "count differs from the symbolic step");
    PB_TRY(check_batch(count, A, B));
    if (!C) return fail(PB_ERR_ARG, "C is NULL");
    for (int32_t i = 0; i < count; ++i) {
        const ProbDesc &d = p->hdesc[i];
        if (A[i].nrows != d.m || A[i].ncols != d.k || B[i].ncols != d.n || A[i].nnz != d.nnza || B[i].nnz != d.nnzb)
            return fail(PB_ERR_SHAPE, "problem %d differs from the symbolic step", i);
        if (!C[i].rowptr) return fail(PB_ERR_ARG, "C[%d].rowptr is NULL", i);
        if (C[i].capacity < 0) return fail(PB_ERR_SHAPE, "C[%d] has negative capacity", i);
        if (C[i].capacity > 0 && (!C[i].colidx || !C[i].val)) return fail(PB_ERR_ARG, "C[%d].colidx/val is NULL", i);
    }
    if (p->ws_bytes > 0 && (!workspace || workspace_bytes < p->ws_bytes))
        return fail(PB_ERR_WORKSPACE, "numeric workspace has %zu bytes, needs %zu", workspace_bytes, p->ws_bytes);

    hipStream_t st = (hipStream_t)hip_stream;
    NumLayout L = num_layout(workspace, p);
    const int32_t cnt = p->count;
    // The staging area is read by the previous call's uploads, which may
    // still be queued: wait for them before rewriting it.  Under stream
    // capture nothing is waited for or recorded; a replay then uploads what
    // the staging area holds at replay time (the latest call's descriptors).
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    PB_HIP(hipStreamIsCapturing(st, &cap));
    const bool capturing = cap != hipStreamCaptureStatusNone;
    if (!capturing && p->staged_pending) {
        PB_HIP(hipEventSynchronize(p->staged));
        p->staged_pending = false;
    }
    // input descriptors (the arrays may have moved since the symbolic step)
    // and output descriptors, through the pinned staging area
    ProbDesc *sd = staged_desc(p);
    OutDesc *so = staged_outs(p);
    for (int32_t i = 0; i < cnt; ++i) {
        sd[i] = p->hdesc[i];
        if (i < count) {
            sd[i].aptr = A[i].ptr;
            sd[i].aidx = A[i].idx;
            sd[i].aval = A[i].val;
            sd[i].bptr = B[i].ptr;
            sd[i].bidx = B[i].idx;
            sd[i].bval = B[i].val;
            so[i] = OutDesc{C[i].rowptr, C[i].colidx, C[i].val, C[i].capacity, sd[i].mbase, sd[i].m};
        } else {
            so[i] = OutDesc{nullptr, nullptr, nullptr, 0, sd[i].mbase, 0};
        }
    }
    PB_HIP(hipMemcpyAsync(p->pdesc, sd, sizeof(ProbDesc) * cnt, hipMemcpyHostToDevice, st));
    PB_HIP(hipMemcpyAsync(L.outs, so, sizeof(OutDesc) * cnt, hipMemcpyHostToDevice, st));
    if (!capturing) {
        if (!p->staged) PB_HIP(hipEventCreateWithFlags(&p->staged, hipEventDisableTiming));
        PB_HIP(hipEventRecord(p->staged, st));
        p->staged_pending = true;
    }
    PB_TRY(fill_zero(workspace, L.zero_bytes, st));
    PB_TRY(launch_pack(p, 2, st));
    for (int32_t i = 0; i < count; ++i)
        if (p->hdesc[i].m == 0) PB_TRY(fill_zero(C[i].rowptr, sizeof(int64_t), st));
    PB_TRY(run_numeric(p, L, p->acp, p->ari, p->av, p->brp, p->bci, p->bv, nullptr, st));
    if (nnzC) {
        std::vector<int64_t> tot(count, 0);
        uint32_t err = 0;
        for (int32_t i = 0; i < count; ++i)
            PB_HIP(hipMemcpyAsync(&tot[i], C[i].rowptr + p->hdesc[i].m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        PB_HIP(hipMemcpyAsync(&err, L.err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        PB_HIP(hipStreamSynchronize(st));
        if (err & ~(uint32_t)kErrCapacity) return fail(PB_ERR_INTERNAL, "numeric device error 0x%x", err);
        pb_status rs = PB_OK;
        for (int32_t i = 0; i < count; ++i) {
            nnzC[i] = tot[i];
            if (tot[i] > C[i].capacity && rs == PB_OK)
                rs = fail(PB_ERR_CAPACITY, "C[%d] needs %lld entries, capacity %lld", i, (long long)tot[i],
                          (long long)C[i].capacity);
        }
        return rs;
    }
    return PB_OK;
}

pb_status spgemm_plan_info(const pb_plan *p, pb_plan_info *info) {
    if (!p || !info) return fail(PB_ERR_ARG, "NULL argument");
    std::memset(info, 0, sizeof *info);
    info->m = p->m;
    info->k = p->k;
    info->n = p->n;
    info->flop = (int64_t)p->h.flop;
    info->slots = (int64_t)p->h.slots;
    info->run_align = p->align;
    info->row_count = p->rowcount;
    info->deterministic = p->det;
    info->nbins = (int64_t)p->h.nbins;
    info->max_bin_tuples = (int64_t)p->h.maxbin;
    info->max_row_flop = (int64_t)p->h.maxrow;
    info->tile_tuples = p->T;
    info->expand_chunk = p->chunk;
    info->col_bits = p->cb;
    info->precision = (int32_t)p->prec;
    info->count = p->user_count;
    return PB_OK;
}

void spgemm_plan_destroy(pb_plan *p) { delete p; }

pb_status spgemm_profile_begin(void) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    for (auto &r : g_prof.recs) {
        g_prof.pool.push_back(r.e0);
        g_prof.pool.push_back(r.e1);
    }
    g_prof.recs.clear();
    g_prof.on = true;
    return PB_OK;
}

pb_status spgemm_profile_end(pb_profile *out) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = false;
    if (!out) return fail(PB_ERR_ARG, "out is NULL");
    std::memset(out, 0, sizeof *out);
    for (auto &r : g_prof.recs) {
        PB_HIP(hipEventSynchronize(r.e1));
        float ms = 0.f;
        PB_HIP(hipEventElapsedTime(&ms, r.e0, r.e1));
        if (r.phase >= 0 && r.phase < PB_NPHASES) {
            out->ms[r.phase] += ms;
            out->launches[r.phase] += 1;
        }
    }
    return PB_OK;
}

pb_status spgemm_copy(void *dst, const void *src, size_t bytes, void *hip_stream) {
    if (!dst || !src) return fail(PB_ERR_ARG, "NULL pointer");
    if ((bytes & 15) || (((uintptr_t)dst | (uintptr_t)src) & 15)) return fail(PB_ERR_ARG, "16-byte alignment required");
    const int64_t n = (int64_t)(bytes / 16);
    if (n == 0) return PB_OK;
    const int64_t grid = ceil_div(n, 256);
    if (grid > 0x7fffffffll) return fail(PB_ERR_RANGE, "copy too large");
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)hip_stream, (uint4 *)dst,
                       (const uint4 *)src, n);
    PB_LAUNCHED("copy");
    return PB_OK;
}

}  // extern "C"
