// Host runtime of the PB-SpGEMM library: C ABI, validation, workspace
// layout, kernel launches.  See include/pbspgemm.h for the contract.
#include "pbspgemm.h"

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pb_kernels.h"

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

// Kernel shapes.
constexpr int kScanBlock = 256, kScanIpt = 8, kScanTile = kScanBlock * kScanIpt;
constexpr int kSortBlock = 512, kSortTmax = 4096;
constexpr int kSortBlockSmall = 256, kSortTmaxSmall = 2048;
constexpr int kExpBlock = 256, kExpWin = 2048;
constexpr int kDefaultTile = 4096;
constexpr int kDefaultChunk = 4096;

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

pb_status check_csx(const pb_csx *x, const char *name, bool csc) {
    if (!x) return fail(PB_ERR_ARG, "%s is NULL", name);
    if (x->nrows < 0 || x->ncols < 0 || x->nnz < 0) return fail(PB_ERR_SHAPE, "%s has a negative size", name);
    if (x->nrows > kMaxDim || x->ncols > kMaxDim) return fail(PB_ERR_RANGE, "%s dimension exceeds 2^31-1", name);
    if (x->nnz > kMaxCount) return fail(PB_ERR_RANGE, "%s nnz exceeds 2^62", name);
    if (!x->ptr) return fail(PB_ERR_ARG, "%s.ptr is NULL", name);
    if (x->nnz > 0 && (!x->idx || !x->val)) return fail(PB_ERR_ARG, "%s.idx/val is NULL with nnz > 0", name);
    (void)csc;
    return PB_OK;
}

int col_bits(int64_t n) {
    if (n <= 1) return 0;
    return 64 - __builtin_clzll((uint64_t)(n - 1));
}

}  // namespace

// ---- plan ----------------------------------------------------------------
struct pb_plan {
    int64_t m = 0, k = 0, n = 0, nnzA = 0, nnzB = 0;
    pb_precision prec = PB_F64;
    int T = kDefaultTile, chunk = kDefaultChunk, cb = 0;
    // symbolic workspace tables
    SymInfo *info = nullptr;
    int64_t *F = nullptr;
    uint64_t *R = nullptr;
    RowTab *rowtab = nullptr;
    uint32_t *runpos = nullptr;
    int32_t *binrow0 = nullptr;
    int64_t *binoff = nullptr;
    // host facts
    SymInfo h{};
    int64_t nchunks = 0;
    size_t ws_bytes = 0;
};

namespace {

struct SymLayout {
    SymInfo *info;
    uint32_t *tickets;
    uint64_t *stF, *stR, *stB;
    uint64_t *R;
    int64_t *F;
    RowTab *rowtab;
    uint32_t *runpos;
    int32_t *binrow0;
    int64_t *binoff;
    size_t zero_bytes, total;
};

SymLayout sym_layout(void *base, int64_t m, int64_t k, int64_t nnza) {
    Carver cv(base);
    SymLayout L{};
    // zeroed region first
    L.info = cv.take<SymInfo>(1);
    L.tickets = cv.take<uint32_t>(4);
    L.stF = cv.take<uint64_t>(ceil_div(k, kScanTile) + 1);
    L.stR = cv.take<uint64_t>(ceil_div(m, kScanTile) + 1);
    L.stB = cv.take<uint64_t>(ceil_div(m, kScanTile) + 1);
    L.R = cv.take<uint64_t>(m + 1);
    L.zero_bytes = (cv.off + 255) & ~(size_t)255;
    L.F = cv.take<int64_t>(k + 1);
    L.rowtab = cv.take<RowTab>(m);
    L.runpos = cv.take<uint32_t>(nnza);
    L.binrow0 = cv.take<int32_t>(m + 1);
    L.binoff = cv.take<int64_t>(m + 1);
    L.total = (cv.off + 255) & ~(size_t)255;
    return L;
}

struct NumLayout {
    uint32_t *ticket, *err;
    uint64_t *status;
    int32_t *kstart;
    uint32_t *rownnz;
    uint32_t *keys;
    void *vals;
    size_t zero_bytes, total;
};

NumLayout num_layout(void *base, const pb_plan *p) {
    Carver cv(base);
    NumLayout L{};
    L.ticket = cv.take<uint32_t>(2);
    L.err = L.ticket + 1;
    L.status = cv.take<uint64_t>(ceil_div(p->m, kScanTile) + 1);
    L.zero_bytes = (cv.off + 255) & ~(size_t)255;
    L.kstart = cv.take<int32_t>(p->nchunks + 1);
    L.rownnz = cv.take<uint32_t>(p->m);
    const int64_t flop = (int64_t)p->h.flop;
    L.keys = cv.take<uint32_t>(flop);
    if (p->prec == PB_F64) L.vals = cv.take<double>(flop);
    else L.vals = cv.take<float>(flop);
    L.total = (cv.off + 255) & ~(size_t)255;
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

template <class Op, class Src, class Dst>
pb_status launch_scan(int64_t n, Src src, Dst dst, uint64_t *status, uint32_t *ticket, uint32_t *err,
                      hipStream_t st, const char *name) {
    if (n <= 0) return PB_OK;
    const int64_t tiles = ceil_div(n, kScanTile);
    hipLaunchKernelGGL((k_chained_scan<kScanBlock, kScanIpt, Op, Src, Dst>), dim3((unsigned)tiles), dim3(kScanBlock),
                       0, st, n, src, dst, status, ticket, err);
    PB_LAUNCHED(name);
    return PB_OK;
}

// Workgroups of a persistent kernel: as many as fit on the device at once
// (at most `work`, at least 1).
unsigned resident_grid(const void *kern, int block, int64_t work) {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, 0) != hipSuccess || per <= 0) per = 1;
    int64_t g = (int64_t)per * cus;
    if (g > work) g = work;
    return (unsigned)(g > 0 ? g : 1);
}

pb_status resolve_tune(const pb_tune *t, int *T, int *chunk) {
    *T = kDefaultTile;
    *chunk = kDefaultChunk;
    if (!t) return PB_OK;
    if (t->tile_tuples) {
        if (t->tile_tuples < 256 || t->tile_tuples > kSortTmax)
            return fail(PB_ERR_ARG, "tile_tuples must be in [256, %d]", kSortTmax);
        *T = t->tile_tuples;
    }
    if (t->expand_chunk) {
        if (t->expand_chunk != 2048 && t->expand_chunk != 4096)
            return fail(PB_ERR_ARG, "expand_chunk must be 2048 or 4096");
        *chunk = t->expand_chunk;
    }
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

pb_status spgemm_symbolic(const pb_csx *A, const pb_csx *B, pb_precision prec, const pb_tune *tune, void *sym_ws,
                          size_t *sym_ws_bytes, void *hip_stream, pb_plan **plan, int64_t *flop,
                          size_t *workspace_bytes) {
    g_last_error.clear();
    pb_status s;
    if ((s = check_csx(A, "A", true)) != PB_OK) return s;
    if ((s = check_csx(B, "B", false)) != PB_OK) return s;
    if (A->ncols != B->nrows) return fail(PB_ERR_SHAPE, "A.ncols (%lld) != B.nrows (%lld)", (long long)A->ncols, (long long)B->nrows);
    if (prec != PB_F64 && prec != PB_F32C) return fail(PB_ERR_ARG, "unknown precision %d", (int)prec);
    if (!sym_ws_bytes) return fail(PB_ERR_ARG, "sym_ws_bytes is NULL");
    int T, chunk;
    if ((s = resolve_tune(tune, &T, &chunk)) != PB_OK) return s;
    const int64_t m = A->nrows, k = A->ncols, n = B->ncols;
    const size_t need = sym_layout(nullptr, m, k, A->nnz).total;
    if (!sym_ws) {
        *sym_ws_bytes = need;
        return PB_OK;
    }
    if (*sym_ws_bytes < need) return fail(PB_ERR_WORKSPACE, "symbolic workspace has %zu bytes, needs %zu", *sym_ws_bytes, need);
    if (!plan || !flop || !workspace_bytes) return fail(PB_ERR_ARG, "plan/flop/workspace_bytes output is NULL");
    if (B->nnz >= (int64_t)1 << 32) return fail(PB_ERR_RANGE, "nnz(B) must be below 2^32 (32-bit in-row run offsets)");
    const int cb = col_bits(n);
    if (cb > 31) return fail(PB_ERR_RANGE, "n too large for packed keys");

    hipStream_t st = (hipStream_t)hip_stream;
    SymLayout L = sym_layout(sym_ws, m, k, A->nnz);
    pb_plan *p = new pb_plan();
    p->m = m;
    p->k = k;
    p->n = n;
    p->nnzA = A->nnz;
    p->nnzB = B->nnz;
    p->prec = prec;
    p->T = T;
    p->chunk = chunk;
    p->cb = cb;
    p->info = L.info;
    p->F = L.F;
    p->R = L.R;
    p->rowtab = L.rowtab;
    p->runpos = L.runpos;
    p->binrow0 = L.binrow0;
    p->binoff = L.binoff;

    pb_status rs = PB_OK;
    {
        ProfScope ps(st, 0);
        do {
            if ((rs = fill_zero(sym_ws, L.zero_bytes, st)) != PB_OK) break;
            if (k > 0) {
                if ((rs = launch_scan<SumOp>(k, ColFlopSrc{A->ptr, B->ptr}, ColFlopDst{{}, L.F, k, L.info}, L.stF,
                                             &L.tickets[0], &L.info->err, st, "flop scan")) != PB_OK)
                    break;
                const int64_t grid = ceil_div(k, 256);
                hipLaunchKernelGGL(k_rowflop<256>, dim3((unsigned)grid), dim3(256), 0, st, k, A->ptr, A->idx, B->ptr, L.R, L.runpos);
                hipError_t e = hipGetLastError();
                if (e != hipSuccess) { rs = fail(PB_ERR_HIP, "launch rowflop: %s", hipGetErrorString(e)); break; }
            } else {
                if ((rs = fill_zero(L.F, sizeof(int64_t), st)) != PB_OK) break;
            }
            if (m > 0) {
                if ((rs = launch_scan<SumOp>(m, RowFlopSrc{L.R}, RowFlopDst{L.R, m, (uint64_t)(T / 2), L.info}, L.stR,
                                             &L.tickets[1], &L.info->err, st, "row scan")) != PB_OK)
                    break;
                const int rowbits = 32 - cb;
                if ((rs = launch_scan<BinOp>(m, BinSrc{L.R, L.info, (uint64_t)T, rowbits, nullptr, 0},
                                             BinDst{L.rowtab, L.binrow0, L.binoff, L.R, m, (uint64_t)T, L.info},
                                             L.stB, &L.tickets[2], &L.info->err, st, "bin scan")) != PB_OK)
                    break;
            }
        } while (0);
    }
    if (rs != PB_OK) {
        delete p;
        return rs;
    }
    hipError_t e = hipMemcpyAsync(&p->h, L.info, sizeof(SymInfo), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete p;
        return fail(PB_ERR_HIP, "symbolic readback: %s", hipGetErrorString(e));
    }
    if (p->h.err) {
        uint32_t er = p->h.err;
        delete p;
        return fail(PB_ERR_INTERNAL, "symbolic device error 0x%x", er);
    }
    if (m == 0) p->h.nbins = 0;
    if (p->h.noversize) {
        const unsigned long long nov = (unsigned long long)p->h.noversize;
        const long long mr = (long long)p->h.maxrow;
        delete p;
        return fail(PB_ERR_UNSUPPORTED, "%llu rows expand to more than %d tuples (largest %lld); "
                    "bins larger than the LDS tile are not supported", nov, T, mr);
    }
    p->nchunks = ceil_div((int64_t)p->h.flop, chunk);
    p->ws_bytes = num_layout(nullptr, p).total;
    *plan = p;
    *flop = (int64_t)p->h.flop;
    *workspace_bytes = p->ws_bytes;
    return PB_OK;
}

pb_status spgemm_numeric(pb_plan *p, const pb_csx *A, const pb_csx *B, void *workspace, size_t workspace_bytes,
                         pb_csr_out *C, int64_t *nnzC, void *hip_stream) {
    g_last_error.clear();
    if (!p) return fail(PB_ERR_ARG, "plan is NULL");
    pb_status s;
    if ((s = check_csx(A, "A", true)) != PB_OK) return s;
    if ((s = check_csx(B, "B", false)) != PB_OK) return s;
    if (A->nrows != p->m || A->ncols != p->k || B->ncols != p->n || A->nnz != p->nnzA || B->nnz != p->nnzB)
        return fail(PB_ERR_SHAPE, "A/B differ from the matrices given to the symbolic step");
    if (!C || !C->rowptr) return fail(PB_ERR_ARG, "C or C->rowptr is NULL");
    if (C->capacity < 0) return fail(PB_ERR_SHAPE, "negative capacity");
    if (C->capacity > 0 && (!C->colidx || !C->val)) return fail(PB_ERR_ARG, "C->colidx/val is NULL");
    if (p->ws_bytes > 0 && (!workspace || workspace_bytes < p->ws_bytes))
        return fail(PB_ERR_WORKSPACE, "numeric workspace has %zu bytes, needs %zu", workspace_bytes, p->ws_bytes);

    hipStream_t st = (hipStream_t)hip_stream;
    const int64_t flop = (int64_t)p->h.flop;
    const int64_t nbins = (int64_t)p->h.nbins;
    NumLayout L = num_layout(workspace, p);
    if ((s = fill_zero(workspace, L.zero_bytes, st)) != PB_OK) return s;
    if (p->m == 0) {
        if ((s = fill_zero(C->rowptr, sizeof(int64_t), st)) != PB_OK) return s;
    }
    if (flop > 0) {
        const int64_t nthreads = p->nchunks + 1;
        hipLaunchKernelGGL(k_chunk_start, dim3((unsigned)ceil_div(nthreads, 256)), dim3(256), 0, st, p->nchunks,
                           (int64_t)p->chunk, p->k, p->F, L.kstart);
        PB_LAUNCHED("chunk start");
        ExpandArgs ea{flop, p->k, p->F, L.kstart, A->ptr, A->idx, A->val, B->ptr, B->idx, B->val,
                      p->runpos, p->rowtab, L.keys, L.vals, p->cb, L.err};
        ProfScope ps(st, 1);
        if (p->chunk == 4096) {
            if (p->prec == PB_F64)
                hipLaunchKernelGGL((k_expand<kExpBlock, 16, kExpWin, double>), dim3((unsigned)p->nchunks), dim3(kExpBlock), 0, st, ea);
            else
                hipLaunchKernelGGL((k_expand<kExpBlock, 16, kExpWin, float>), dim3((unsigned)p->nchunks), dim3(kExpBlock), 0, st, ea);
        } else {
            if (p->prec == PB_F64)
                hipLaunchKernelGGL((k_expand<kExpBlock, 8, kExpWin, double>), dim3((unsigned)p->nchunks), dim3(kExpBlock), 0, st, ea);
            else
                hipLaunchKernelGGL((k_expand<kExpBlock, 8, kExpWin, float>), dim3((unsigned)p->nchunks), dim3(kExpBlock), 0, st, ea);
        }
        PB_LAUNCHED("expand");
    }
    if (nbins > 0) {
        {
            ProfScope ps(st, 3);
            CountArgs ca{p->binrow0, p->binoff, L.keys, p->cb, L.rownnz, L.err};
            if (p->T <= kSortTmaxSmall)
                hipLaunchKernelGGL((k_row_nnz<512, kSortTmaxSmall>), dim3((unsigned)nbins), dim3(512), 0, st, ca);
            else
                hipLaunchKernelGGL((k_row_nnz<512, kSortTmax>), dim3((unsigned)nbins), dim3(512), 0, st, ca);
            PB_LAUNCHED("row counts");
            if ((s = launch_scan<SumOp>(p->m, RowNnzSrc{L.rownnz}, RowPtrDst{{}, C->rowptr, p->m}, L.status, L.ticket,
                                        L.err, st, "row pointer scan")) != PB_OK)
                return s;
        }
        SortArgs sa{p->binrow0, p->binoff, L.keys, L.vals, p->cb, L.err, C->rowptr, C->colidx, C->val, C->capacity};
        ProfScope ps(st, 2);
        if (p->T <= kSortTmaxSmall) {
            if (p->prec == PB_F64)
                hipLaunchKernelGGL((k_sort_compress<kSortBlockSmall, kSortTmaxSmall, double>), dim3((unsigned)nbins), dim3(kSortBlockSmall), 0, st, sa);
            else
                hipLaunchKernelGGL((k_sort_compress<kSortBlockSmall, kSortTmaxSmall, float>), dim3((unsigned)nbins), dim3(kSortBlockSmall), 0, st, sa);
        } else {
            if (p->prec == PB_F64)
                hipLaunchKernelGGL((k_sort_compress<kSortBlock, kSortTmax, double>), dim3((unsigned)nbins), dim3(kSortBlock), 0, st, sa);
            else
                hipLaunchKernelGGL((k_sort_compress<kSortBlock, kSortTmax, float>), dim3((unsigned)nbins), dim3(kSortBlock), 0, st, sa);
        }
        PB_LAUNCHED("sort+compress");
    }
    if (nnzC) {
        int64_t total = 0;
        uint32_t err = 0;
        PB_HIP(hipMemcpyAsync(&total, C->rowptr + p->m, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        PB_HIP(hipMemcpyAsync(&err, L.err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
        PB_HIP(hipStreamSynchronize(st));
        *nnzC = total;
        if (err & ~(uint32_t)kErrCapacity) return fail(PB_ERR_INTERNAL, "numeric device error 0x%x", err);
        if ((err & kErrCapacity) || total > C->capacity)
            return fail(PB_ERR_CAPACITY, "C needs %lld entries, capacity %lld", (long long)total, (long long)C->capacity);
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
    info->nbins = (int64_t)p->h.nbins;
    info->max_bin_tuples = -1;
    info->max_row_flop = (int64_t)p->h.maxrow;
    info->tile_tuples = p->T;
    info->expand_chunk = p->chunk;
    info->col_bits = p->cb;
    info->precision = (int32_t)p->prec;
    info->count = 1;
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
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)hip_stream, (uint4 *)dst, (const uint4 *)src, n);
    PB_LAUNCHED("copy");
    return PB_OK;
}

}  // extern "C"
