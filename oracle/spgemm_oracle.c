/*
 * CPU oracle for sparse C = A * B -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code with the GPU path.
 *
 * What it computes (paper, Section 2.1 "Notations" and 2.2): C = A*B where
 * A is m x k stored by columns (CSC) and B is k x n stored by rows (CSR).
 * The expanded matrix C^ holds one tuple per multiplication
 * A(r,kk) * B(kk,j); C is C^ with tuples of equal (row, col) merged by
 * addition.  An output position is structural when at least one tuple lands
 * on it, so a sum that cancels to 0.0 is still a stored entry.
 *
 * Method (Gustavson's column formulation, Section 2.2, Fig. 1): column j of
 * C gathers, for every kk in B(:,j) in ascending kk order and every r in
 * A(:,kk) in ascending r order, the tuple (r, A(r,kk)*B(kk,j)); the list is
 * stably sorted by r and every run of equal r is summed left to right in
 * double precision.  Hence each C(r,j) is the sum over ascending kk of the
 * rounded products, added one at a time.  Build with -ffp-contract=off so no
 * multiply-add is fused.
 *
 * Alongside the value, N(r,j) = sum |A(r,kk)| * |B(kk,j)| is returned: the
 * usual normaliser for the forward error of a dot product with signed terms.
 *
 * The flop count is the paper's symbolic count (Algorithm 3):
 *   flop = sum over kk of nnz(A(:,kk)) * nnz(B(kk,:)),
 * multiplications only.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

typedef struct {
    int32_t row;
    double val;
    double absval;
} tuple_t;

/* Stable bottom-up merge sort of tuples by row. */
static void merge_sort_by_row(tuple_t *a, tuple_t *tmp, int64_t n)
{
    tuple_t *src = a, *dst = tmp;
    for (int64_t width = 1; width < n; width *= 2) {
        for (int64_t lo = 0; lo < n; lo += 2 * width) {
            int64_t mid = lo + width < n ? lo + width : n;
            int64_t hi = lo + 2 * width < n ? lo + 2 * width : n;
            int64_t i = lo, j = mid, o = lo;
            while (i < mid && j < hi) {
                /* take from the left run on ties: stability */
                if (src[j].row < src[i].row) dst[o++] = src[j++];
                else dst[o++] = src[i++];
            }
            while (i < mid) dst[o++] = src[i++];
            while (j < hi) dst[o++] = src[j++];
        }
        tuple_t *t = src; src = dst; dst = t;
    }
    if (src != a) memcpy(a, src, (size_t)n * sizeof(tuple_t));
}

int64_t oracle_flop(int64_t k, const int64_t *a_colptr, const int64_t *b_rowptr)
{
    int64_t flop = 0;
    for (int64_t kk = 0; kk < k; ++kk)
        flop += (a_colptr[kk + 1] - a_colptr[kk]) * (b_rowptr[kk + 1] - b_rowptr[kk]);
    return flop;
}

/* Stable counting-sort transpose of compressed storage: the input has
 * nmajor slices over nminor indices; the output has nminor slices holding
 * the former major indices in ascending order. */
int oracle_transpose(int64_t nmajor, int64_t nminor, const int64_t *ptr, const int32_t *idx,
                     const double *val, int64_t *tptr, int32_t *tidx, double *tval)
{
    int64_t nnz = ptr[nmajor];
    int64_t *cursor = (int64_t *)calloc((size_t)nminor + 1, sizeof(int64_t));
    if (!cursor) return 1;
    for (int64_t p = 0; p < nnz; ++p) cursor[idx[p] + 1]++;
    for (int64_t i = 0; i < nminor; ++i) cursor[i + 1] += cursor[i];
    memcpy(tptr, cursor, (size_t)(nminor + 1) * sizeof(int64_t));
    for (int64_t s = 0; s < nmajor; ++s) {
        for (int64_t p = ptr[s]; p < ptr[s + 1]; ++p) {
            int64_t q = cursor[idx[p]]++;
            tidx[q] = (int32_t)s;
            if (val) tval[q] = val[p];
        }
    }
    free(cursor);
    return 0;
}

typedef struct {
    int32_t *idx;
    double *val, *absval;
    int64_t len, cap;
} outbuf_t;

static int outbuf_push(outbuf_t *o, int32_t i, double v, double av)
{
    if (o->len == o->cap) {
        int64_t nc = o->cap ? 2 * o->cap : 1024;
        int32_t *ni = (int32_t *)realloc(o->idx, (size_t)nc * sizeof(int32_t));
        if (!ni) return 1;
        o->idx = ni;
        double *nv = (double *)realloc(o->val, (size_t)nc * sizeof(double));
        if (!nv) return 1;
        o->val = nv;
        double *na = (double *)realloc(o->absval, (size_t)nc * sizeof(double));
        if (!na) return 1;
        o->absval = na;
        o->cap = nc;
    }
    o->idx[o->len] = i;
    o->val[o->len] = v;
    o->absval[o->len] = av;
    o->len++;
    return 0;
}

/*
 * Selected columns of C = A * B.
 *   A: m x k, CSC (a_colptr[k+1], a_rowidx, a_val)
 *   B: k x n, CSR (b_rowptr[k+1], b_colidx, b_val)
 *   cols: nsel column ids in any order (NULL = all n columns, nsel = n)
 * Output (malloc'd, release with oracle_free): for the selected columns in
 * the given order, out_ptr[nsel+1], out_idx / out_val / out_abs[out_ptr[nsel]]
 * with rows ascending in each column.  Returns 0 on success.
 */
int oracle_spgemm_cols(int64_t m, int64_t k, int64_t n,
                       const int64_t *a_colptr, const int32_t *a_rowidx, const double *a_val,
                       const int64_t *b_rowptr, const int32_t *b_colidx, const double *b_val,
                       int64_t nsel, const int64_t *cols, int nthreads,
                       int64_t **out_ptr, int32_t **out_idx, double **out_val, double **out_abs)
{
    (void)m;
    int64_t nnzb = b_rowptr[k];
    /* B by columns: B(:,j) lists (kk, B(kk,j)) with kk ascending. */
    int64_t *bt_ptr = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    int32_t *bt_idx = (int32_t *)malloc((size_t)(nnzb ? nnzb : 1) * sizeof(int32_t));
    double *bt_val = (double *)malloc((size_t)(nnzb ? nnzb : 1) * sizeof(double));
    if (!bt_ptr || !bt_idx || !bt_val) return 1;
    if (oracle_transpose(k, n, b_rowptr, b_colidx, b_val, bt_ptr, bt_idx, bt_val)) return 1;

    if (nthreads <= 0) nthreads = omp_get_max_threads();
    if (nsel < nthreads) nthreads = nsel > 0 ? (int)nsel : 1;
    outbuf_t *bufs = (outbuf_t *)calloc((size_t)nthreads, sizeof(outbuf_t));
    int64_t *counts = (int64_t *)calloc((size_t)nsel + 1, sizeof(int64_t));
    int failed = 0;

#pragma omp parallel num_threads(nthreads)
    {
        int tid = omp_get_thread_num();
        int nt = omp_get_num_threads();
        int64_t s0 = nsel * tid / nt, s1 = nsel * (tid + 1) / nt;
        int64_t cap = 0;
        tuple_t *work = NULL, *tmp = NULL;
        outbuf_t *o = &bufs[tid];
        for (int64_t s = s0; s < s1 && !failed; ++s) {
            int64_t j = cols ? cols[s] : s;
            /* gather the column's tuples: kk ascending, then r ascending */
            int64_t len = 0;
            for (int64_t q = bt_ptr[j]; q < bt_ptr[j + 1]; ++q) {
                int64_t kk = bt_idx[q];
                len += a_colptr[kk + 1] - a_colptr[kk];
            }
            if (len > cap) {
                cap = len * 2;
                free(work); free(tmp);
                work = (tuple_t *)malloc((size_t)cap * sizeof(tuple_t));
                tmp = (tuple_t *)malloc((size_t)cap * sizeof(tuple_t));
                if (!work || !tmp) { failed = 1; break; }
            }
            int64_t w = 0;
            for (int64_t q = bt_ptr[j]; q < bt_ptr[j + 1]; ++q) {
                int64_t kk = bt_idx[q];
                double bv = bt_val[q];
                for (int64_t p = a_colptr[kk]; p < a_colptr[kk + 1]; ++p) {
                    double prod = a_val[p] * bv;
                    work[w].row = a_rowidx[p];
                    work[w].val = prod;
                    work[w].absval = fabs(a_val[p]) * fabs(bv);
                    w++;
                }
            }
            merge_sort_by_row(work, tmp, len);
            int64_t before = o->len;
            for (int64_t i = 0; i < len;) {
                int32_t r = work[i].row;
                double sum = work[i].val, asum = work[i].absval;
                int64_t t = i + 1;
                while (t < len && work[t].row == r) {
                    sum = sum + work[t].val;
                    asum = asum + work[t].absval;
                    t++;
                }
                if (outbuf_push(o, r, sum, asum)) { failed = 1; break; }
                i = t;
            }
            counts[s + 1] = o->len - before;
        }
        free(work);
        free(tmp);
    }
    free(bt_ptr); free(bt_idx); free(bt_val);
    if (failed) return 1;

    int64_t *ptr = (int64_t *)malloc((size_t)(nsel + 1) * sizeof(int64_t));
    ptr[0] = 0;
    for (int64_t s = 0; s < nsel; ++s) ptr[s + 1] = ptr[s] + counts[s + 1];
    int64_t total = ptr[nsel];
    int32_t *idx = (int32_t *)malloc((size_t)(total ? total : 1) * sizeof(int32_t));
    double *val = (double *)malloc((size_t)(total ? total : 1) * sizeof(double));
    double *abv = (double *)malloc((size_t)(total ? total : 1) * sizeof(double));
    int64_t off = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (bufs[t].len) {
            memcpy(idx + off, bufs[t].idx, (size_t)bufs[t].len * sizeof(int32_t));
            memcpy(val + off, bufs[t].val, (size_t)bufs[t].len * sizeof(double));
            memcpy(abv + off, bufs[t].absval, (size_t)bufs[t].len * sizeof(double));
        }
        off += bufs[t].len;
        free(bufs[t].idx); free(bufs[t].val); free(bufs[t].absval);
    }
    free(bufs);
    free(counts);
    *out_ptr = ptr;
    *out_idx = idx;
    *out_val = val;
    *out_abs = abv;
    return 0;
}

void oracle_free(void *p) { free(p); }

int oracle_max_threads(void) { return omp_get_max_threads(); }
