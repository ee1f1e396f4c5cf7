/*
 * pbspgemm.h -- C ABI of the MI355X (gfx950) PB-SpGEMM library.
 *
 * Computes C = A * B for sparse A (m x k, CSC) and B (k x n, CSR) and emits
 * C in CSR, by the outer-product expand-sort-compress method with
 * propagation blocking of Gu, Moreira, Edelsohn and Azad (arXiv 2002.11302):
 *
 *   symbolic  -- Algorithm 3 (flop = sum_k nnz(A(:,k)) * nnz(B(k,:))), extended
 *                with the per-row flop count the paper sketches beside it, to
 *                cut the rows of C into bins of consecutive rows whose
 *                tuples fit one workgroup's LDS tile (Section 3.2, and the
 *                variable row ranges of Section 3.4);
 *   expand    -- Algorithm 2's outer-product loop: every product
 *                A(r,k) * B(k,c) becomes a tuple appended to the bin of row r
 *                (Section 3.3);
 *   sort      -- per-bin sort in LDS on a packed 32-bit (row-in-bin, column)
 *                key (Section 3.4): a bucket sort, or an LSD radix sort
 *                when the keys cluster;
 *   compress  -- per-bin merge of equal keys by addition (Section 3.5);
 *   ConvertCSR-- entries per row from a key-only count pass, row pointers
 *                from a scan over the rows, then every bin writes its rows
 *                at their final places (Algorithm 2, last step).
 *
 * Conventions for every entry point
 *   - All matrix arrays are DEVICE pointers owned by the caller.  The library
 *     never allocates device memory: scratch space comes in caller-provided
 *     workspaces whose sizes the library reports.
 *   - Index arrays are int32, pointer arrays int64, input values double.
 *     Inside each column of A / row of B indices strictly increase; ptr[0]
 *     is 0 and ptr[end] equals nnz.  These array contents are trusted (they
 *     live on the device); shapes, sizes and null pointers are checked on
 *     the host before any launch.
 *   - Stored zeros in A or B are structural, and an output entry whose sum
 *     cancels to 0.0 stays stored (C keeps every position hit by a product).
 *   - `hip_stream` is a hipStream_t (NULL = default stream).  Work is
 *     stream-ordered; an entry point synchronises only where stated.
 *   - Errors are returned as pb_status; nothing aborts or throws across the
 *     ABI.  spgemm_last_error() gives a thread-local detail string.
 */
#ifndef PBSPGEMM_H
#define PBSPGEMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PB_OK = 0,
    PB_ERR_ARG = 1,         /* null pointer, bad enum, bad tuning value */
    PB_ERR_SHAPE = 2,       /* A.ncols != B.nrows, negative sizes, nnz mismatch with capacity */
    PB_ERR_RANGE = 3,       /* a dimension >= 2^31, or counts beyond 2^62 */
    PB_ERR_WORKSPACE = 4,   /* workspace pointer null or smaller than reported */
    PB_ERR_CAPACITY = 5,    /* C.capacity < nnz(C); *nnzC receives the size needed */
    PB_ERR_HIP = 6,         /* a HIP runtime call failed (detail in spgemm_last_error) */
    PB_ERR_UNSUPPORTED = 7, /* a case the library does not handle (detail in spgemm_last_error) */
    PB_ERR_INTERNAL = 8     /* a device-side consistency check failed */
} pb_status;

typedef enum {
    PB_F64 = 0,  /* tuples and C values in double; sums in double */
    PB_F32C = 1  /* tuples carry fl32(a*b) (product in double, rounded once);
                    each output is a compensated (Neumaier) float sum, or a
                    double sum rounded once where a bin or column window is
                    summed by accumulation; C values float */
} pb_precision;

/* A compressed sparse matrix.  For CSC, ptr has ncols+1 entries and idx
 * holds row indices; for CSR, ptr has nrows+1 entries and idx holds column
 * indices. */
typedef struct {
    int64_t nrows, ncols, nnz;
    const int64_t *ptr;
    const int32_t *idx;
    const double *val;
} pb_csx;

/* Output C in CSR.  rowptr has nrows(C)+1 entries; colidx / val have room
 * for `capacity` entries (nnz(C) <= flop, so capacity = flop always fits).
 * val is double* for PB_F64 and float* for PB_F32C. */
typedef struct {
    int64_t *rowptr;
    int32_t *colidx;
    void *val;
    int64_t capacity;
} pb_csr_out;

/* Tuning knobs; 0 selects the default.  PB_TUNE in the environment
 * ("key=value" pairs separated by ',' or ';', keys named as the fields
 * below, e.g. PB_TUNE="tile_tuples=4096,expand_chunk=512") fills the fields
 * a call leaves at 0 (also when tune is NULL); a malformed PB_TUNE or an
 * unknown key makes the symbolic calls return PB_ERR_ARG.
 *   tile_tuples   upper bound on tuples per bin (LDS sort tile): 256..4096;
 *                 default 2048 for a single product, 4096 for a batch
 *   expand_chunk  tuples per expand wave: 256, 512, 1024 or 2048
 *   round_tuples  upper bound on tuple slots per round (0 = no bound): the
 *                 rows of C are cut into rounds of consecutive bins so that
 *                 one round's tuples fit the workspace (a single bin larger
 *                 than the bound is a round by itself)
 *   run_align     slots per run are rounded up to a multiple of this (1, 4
 *                 or 8; 0 = 4 for PB_F64 when nnz(B) >= 12 * B.nrows, else 1).  The
 *                 tuples of one A entry (a run) then start on a 32-byte
 *                 sector of the tuple arrays, so runs written by different
 *                 waves never share a sector; padding slots carry a sentinel
 *                 key.  Batched plans always use 1.
 *   row_count     how the symbolic step counts tuples per row of C and
 *                 places each A entry's run inside its row: 1 = one device
 *                 atomic per entry of A; 2 = row buckets (the entries of A
 *                 are first distributed to buckets of 4096 consecutive rows
 *                 by a counting sort, then each bucket counts in LDS; needs
 *                 0 < nnz(A) < 2^32 and at most 2^25 rows, else PB_ERR_ARG);
 *                 0 = 2 when it applies, else 1.  C is the same either way
 *                 up to the order in which equal positions are summed.
 *   convert       how C's row pointers are formed (ConvertCSR): 1 = a
 *                 key-only count pass gives the entries of every row and a
 *                 scan over the rows gives the pointers, before the sort;
 *                 2 = fused into the sort (each bin counts its distinct keys
 *                 and takes the entries before it from the earlier bins by a
 *                 decoupled look-back over bins taken in ticket order;
 *                 measured slower: the bins' tickets, all taken from one
 *                 device-wide counter, serialise); 0 = 1.  C is
 *                 the same either way.
 *   deterministic 1 = bit-identical C on every call with the same inputs and
 *                 tuning (Section 3.4's bins summed in a fixed order): the
 *                 runs of a row of C sit in ascending column order of A, the
 *                 bin sort is stable, and every entry of C is summed one
 *                 tuple at a time in that order, so an FP64 entry is
 *                 ((A(i,k1)B(k1,j) + A(i,k2)B(k2,j)) + ...) over ascending k,
 *                 rounded after every operation.  Costs a per-row ordering
 *                 pass in the symbolic step and gives up the LDS hash
 *                 pre-summation and the segmented reduction.  Needs row
 *                 buckets (see row_count; row_count 1 is PB_ERR_ARG),
 *                 convert 0 or 1 (2 is PB_ERR_ARG), and no row of C wider than
 *                 the tile (the symbolic step returns PB_ERR_UNSUPPORTED).
 *                 Batched plans follow it too.  0 = off. */
typedef struct {
    int32_t tile_tuples;
    int32_t expand_chunk;
    int64_t round_tuples;
    int32_t run_align;
    int32_t row_count;
    int32_t convert;
    int32_t deterministic;
} pb_tune;

/* Plan facts (host copy, filled by the symbolic step). */
typedef struct {
    int64_t m, k, n;          /* C is m x n, inner dimension k */
    int64_t flop;             /* multiplications = number of expanded tuples */
    int64_t nbins;            /* bins of consecutive rows */
    int64_t max_bin_tuples;   /* tuple slots of the largest bin (a wide row is a bin by itself) */
    int64_t max_row_flop;     /* largest row of C^ */
    int32_t tile_tuples, expand_chunk;
    int32_t col_bits;         /* bits of the column part of a packed key */
    int32_t precision;        /* pb_precision */
    int64_t count;            /* problems in the plan (1 unless batched) */
    int64_t slots;            /* tuple slots (flop plus run padding) */
    int32_t run_align;        /* run alignment in slots */
    int32_t row_count;        /* 1 device atomics, 2 row buckets (see pb_tune) */
    int32_t deterministic;    /* 1 if the plan sums in the fixed order (see pb_tune) */
    int32_t reserved;
} pb_plan_info;

typedef struct pb_plan pb_plan; /* opaque, host-side */

/*
 * Symbolic step (Algorithm 3 plus the bin cut).
 *
 * prec is a pb_precision value (PB_F64 or PB_F32C), passed as a plain
 * 32-bit integer so that any value a caller passes is defined behaviour;
 * others are PB_ERR_ARG.
 *
 * Size query: with sym_ws == NULL, writes the symbolic workspace size to
 * *sym_ws_bytes and returns PB_OK without touching the device.
 *
 * Otherwise sym_ws must hold *sym_ws_bytes bytes of device memory; it keeps
 * the bin tables and must stay alive, unmodified, until the plan's last
 * numeric call has completed.  The call launches the flop scan, the per-row
 * flop count and the bin cut on hip_stream, then synchronises the stream
 * once to read the totals.  On success *plan is a new host-side plan (free it
 * with spgemm_plan_destroy), *flop the multiplication count and
 * *workspace_bytes the device workspace spgemm_numeric needs.
 */
pb_status spgemm_symbolic(const pb_csx *A_csc, const pb_csx *B_csr, int32_t prec,
                          const pb_tune *tune, void *sym_ws, size_t *sym_ws_bytes,
                          void *hip_stream, pb_plan **plan, int64_t *flop,
                          size_t *workspace_bytes);

/*
 * Operand content.  The kernels trust the operands to be well formed: ptr[0]
 * = 0, ptr non-decreasing, ptr[major] = nnz, indices inside the matrix and
 * strictly increasing within each column (A) or row (B); a malformed operand
 * can make them read or write out of bounds.  With PB_VALIDATE=1 in the
 * environment, spgemm_symbolic and spgemm_batched_symbolic copy every
 * operand's ptr and idx arrays to the host (stream-ordered) and check them
 * before any launch, returning PB_ERR_ARG with the first violation in
 * spgemm_last_error().
 */

/*
 * Rows wider than the tile.  A row of C whose tuples exceed tile_tuples is
 * split after the expand into windows of consecutive columns (2^12 columns
 * while n <= 2^22); windows are binned and sorted and compressed like rows,
 * in bins of at most min(tile_tuples, 2048) tuples, and a window with more
 * tuples than that is summed in LDS by a dense accumulator (tuples added in
 * double; FP32C rounds the double sum to float).  A window that exceeds the
 * tile while being wider than 2^12 columns (n > 2^22 and heavily clustered
 * columns) makes the numeric step return PB_ERR_UNSUPPORTED.
 *
 * Numeric step (Algorithm 2: expand into bins, sort and compress each bin,
 * ConvertCSR).  A_csc / B_csr must be the matrices given to the symbolic
 * step (same arrays and contents).  workspace holds at least the reported
 * bytes; its contents need no initialisation and are scratch afterwards.
 * C->rowptr receives m+1 entries; C->colidx / C->val receive nnz(C)
 * entries.  If nnzC is non-NULL the stream is synchronised and *nnzC is set
 * (PB_ERR_CAPACITY if C->capacity was too small: then only the first
 * `capacity` entries were written and *nnzC is the size needed).  With
 * nnzC == NULL nothing synchronises; nnz(C) is then C->rowptr[m] on the
 * device once the stream reaches this point.
 */
pb_status spgemm_numeric(pb_plan *plan, const pb_csx *A_csc, const pb_csx *B_csr,
                         void *workspace, size_t workspace_bytes, pb_csr_out *C,
                         int64_t *nnzC, void *hip_stream);

/*
 * Numeric step that allocates nothing and takes no workspace: for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  Same contract as
 * spgemm_numeric, except that the numeric workspace is a device array
 * inside the library of PB_NOALLOC_SCRATCH_BYTES bytes, one per GPU, held
 * until the process ends (the GPU is the current device; hip_stream must
 * belong to it).  A plan whose reported workspace_bytes exceed that size is
 * rejected with PB_ERR_WORKSPACE before any launch.  The call makes no
 * hipMalloc / hipFree or other allocating call.  Every call on one GPU uses
 * the same array, and the array keeps the last call's contents (the call
 * clears what must start at zero itself): calls that overlap on one GPU
 * (other host threads, or other streams not ordered with this one) race.
 */
#define PB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
pb_status spgemm_numeric_noalloc(pb_plan *plan, const pb_csx *A_csc, const pb_csx *B_csr, pb_csr_out *C,
                                 int64_t *nnzC, void *hip_stream);

/*
 * Row-range rounds (the paper's partitioned formulation for products whose
 * expanded tuples exceed memory, Sections 2.2 and 3.4).  A plan built with
 * tune->round_tuples > 0 and more tuples than that, or with rows wider than
 * the tile, runs as rounds of consecutive rows.  spgemm_numeric then runs
 * every round in turn into one C (the workspace is reused); the calls below
 * let a caller take C one round at a time instead, when all of C does not
 * fit.  Plans of one round report one round covering every row.
 *
 * spgemm_plan_rounds: *nrounds receives the number of rounds; row_begin
 * (nrounds+1 entries, may be NULL) the first row of each round and m at the
 * end; flop_per_round (nrounds entries, may be NULL) each round's tuples,
 * which bound its nnz(C).  Pass NULL arrays first to learn nrounds.
 *
 * spgemm_numeric_round: computes rows [row_begin[r], row_begin[r+1]) of C
 * into C, whose rowptr then has row_begin[r+1]-row_begin[r]+1 entries
 * starting at 0 and whose colidx / val hold that round's entries.  Same
 * workspace, synchronisation and error rules as spgemm_numeric.
 */
pb_status spgemm_plan_rounds(const pb_plan *plan, int64_t *nrounds, int64_t *row_begin, int64_t *flop_per_round);
pb_status spgemm_numeric_round(pb_plan *plan, const pb_csx *A_csc, const pb_csx *B_csr, int64_t round,
                               void *workspace, size_t workspace_bytes, pb_csr_out *C, int64_t *nnzC,
                               void *hip_stream);

/*
 * Batched products C_i = A_i * B_i, i < count, of uneven sizes (a workload
 * beyond the paper).  The batch runs as one block-diagonal product: the
 * problems' rows and inner indices are laid side by side, bins never span
 * two problems, and every kernel of the path is launched once for the whole
 * batch.  A_csc / B_csr / C are arrays of `count` descriptors.
 *
 * spgemm_batched_symbolic: as spgemm_symbolic (size query with
 * sym_ws == NULL; one stream sync otherwise); `flop` is a host array of
 * `count` entries that receives each problem's multiplication count (the
 * capacity that always fits its C).  The symbolic workspace also holds a
 * packed copy of the inputs' structure.
 *
 * spgemm_batched: the numeric step for the whole batch.  C[i].rowptr gets
 * A_i.nrows+1 entries.  With nnzC == NULL nothing synchronises and the call
 * only enqueues work on hip_stream (descriptor uploads from pinned memory
 * owned by the plan, then kernels), so it can be captured in a hipGraph and
 * replayed while the plan and the descriptor arrays' contents are unchanged;
 * otherwise nnzC is a host array of `count` entries (PB_ERR_CAPACITY names
 * the first problem whose capacity was too small).  The pinned staging area
 * is rewritten by every call: a call first waits (on the host) until the
 * previous call's uploads from it are done, so calls on one plan may be
 * enqueued back to back with different outputs.  Under stream capture that
 * wait is skipped, and a replay uploads what the staging area holds at
 * replay time, i.e. the descriptors of the latest call on the plan: capture
 * after the last eager call on the plan, or keep a plan per captured graph.
 */
pb_status spgemm_batched_symbolic(int32_t count, const pb_csx *A_csc, const pb_csx *B_csr, int32_t prec,
                                  const pb_tune *tune, void *sym_ws, size_t *sym_ws_bytes, void *hip_stream,
                                  pb_plan **plan, int64_t *flop, size_t *workspace_bytes);
pb_status spgemm_batched(pb_plan *plan, int32_t count, const pb_csx *A_csc, const pb_csx *B_csr, void *workspace,
                         size_t workspace_bytes, pb_csr_out *C, int64_t *nnzC, void *hip_stream);

/* Copy the plan's facts to *info. */
pb_status spgemm_plan_info(const pb_plan *plan, pb_plan_info *info);

void spgemm_plan_destroy(pb_plan *plan);
const char *spgemm_status_string(pb_status s);
const char *spgemm_last_error(void);

/* ---------------- measurement support ----------------
 * Kernel timing with HIP events recorded on the launch stream around the
 * library's own kernels.  Phases: 0 symbolic (all its kernels), 1 expand
 * (with a round's restriction of A's columns), 2 sort+compress (and the
 * dense windows' output), 3 entries per row of C and the row-pointer scan,
 * 4 the partition of wide rows into column windows.
 * spgemm_profile_begin clears the accumulators and turns recording on;
 * spgemm_profile_end waits for the recorded events, turns recording off and
 * returns, per phase, the summed milliseconds and the number of launches. */
#define PB_NPHASES 5
typedef struct {
    double ms[PB_NPHASES];
    int64_t launches[PB_NPHASES];
} pb_profile;
pb_status spgemm_profile_begin(void);
pb_status spgemm_profile_end(pb_profile *out);

/* Streaming device copy of `bytes` bytes (16-byte aligned pointers, bytes a
 * multiple of 16): the bandwidth reference (STREAM Copy analogue of the
 * paper's Section 4.2) and the calibration kernel for HBM byte counters. */
pb_status spgemm_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* PBSPGEMM_H */
