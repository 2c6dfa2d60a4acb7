/*
 * CPU oracle for the sparse product C = A * B (CSR, sorted columns).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links, loads or calls
 * this file; only the test-suite, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code with the GPU path.
 *
 * What it computes (OpSparse, Section 2.1, Eq. 1 and Eq. 2):
 *   C_ij = sum_k A_ik * B_kj, evaluated row by row as
 *   C_i* = sum over k in A_i* of A_ik * B_k*   (row-wise / Gustavson dataflow).
 * Structure is the *structural* product of the two patterns (Section 2.2:
 * row sizes come from the indices alone), so an entry whose sum is exactly
 * 0.0 is still stored.  Columns of every output row are ascending (CSR,
 * Section 2.1.1).
 *
 * Method: dense accumulator indexed by column with a "last row that touched
 * this column" marker, plus the list of touched columns, sorted at the end
 * of the row with the C library's qsort.  Products are summed in ascending
 * k (A rows are sorted), then in B-row order, each product rounded to double
 * before the add (build with -ffp-contract=off so no fused multiply-add
 * merges the two roundings).  Alongside each value it accumulates
 * S_ij = sum_k |A_ik * B_kj|, the scale that bounds the rounding error of
 * any summation order.
 *
 * Rows are independent (Section 2.1), so the *_mt entry points run the very
 * same per-row functions on several threads, each with its own accumulator
 * and taking blocks of rows from a shared counter; each row's output goes
 * to its own place, so the result is bit-identical to the single-threaded
 * call.
 *
 * Extra per-row quantities used by the method's setup step (Section 5,
 * setup) and the row-size predictor's features:
 *   n_prod_i = sum over k in A_i* of len(B_k*)   (intermediate products)
 *   a_len_i  = len(A_i*)
 *   b_max_i  = max over k in A_i* of len(B_k*)
 *
 * All index arrays: rpt int64 (absolute offsets; rpt[0] need not be 0),
 * col int32, val double.  Return value 0 on success, negative on bad input
 * or allocation failure.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>

static int cmp_i32(const void *x, const void *y)
{
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    return (a > b) - (a < b);
}

/* Per-row setup quantities.  Any output pointer may be NULL.  Returns the
 * total number of intermediate products. */
int64_t oracle_row_stats(int64_t M, const int64_t *arpt, const int32_t *acol,
                         const int64_t *brpt, int64_t *nprod, int64_t *alen,
                         int64_t *bmax)
{
    int64_t total = 0;
    for (int64_t i = 0; i < M; ++i) {
        int64_t s = 0, mx = 0;
        for (int64_t p = arpt[i]; p < arpt[i + 1]; ++p) {
            int64_t k = acol[p];
            int64_t len = brpt[k + 1] - brpt[k];
            s += len;
            if (len > mx) mx = len;
        }
        if (nprod) nprod[i] = s;
        if (alen) alen[i] = arpt[i + 1] - arpt[i];
        if (bmax) bmax[i] = mx;
        total += s;
    }
    return total;
}

/* Everything one row of either step reads. */
typedef struct {
    int64_t nr;
    const int64_t *rows;
    int64_t N;
    const int64_t *arpt;
    const int32_t *acol;
    const double *aval;
    const int64_t *brpt;
    const int32_t *bcol;
    const double *bval;
    const int64_t *off;     /* numeric: output offsets of the listed rows */
    int64_t *nnz;           /* symbolic: output counts */
    int32_t *ccol;
    double *cval;
    double *cabs;
} job_t;

/* Accumulator of one thread. */
typedef struct {
    int64_t *mark;
    double *acc;
    double *absacc;
    int32_t *list;
} work_t;

static void work_free(work_t *w)
{
    free(w->mark); free(w->acc); free(w->absacc); free(w->list);
    memset(w, 0, sizeof(*w));
}

static int work_init(work_t *w, int64_t N, int numeric)
{
    size_t n = (size_t)(N > 0 ? N : 1);
    memset(w, 0, sizeof(*w));
    w->mark = (int64_t *)malloc(sizeof(int64_t) * n);
    if (numeric) {
        w->acc = (double *)malloc(sizeof(double) * n);
        w->absacc = (double *)malloc(sizeof(double) * n);
        w->list = (int32_t *)malloc(sizeof(int32_t) * n);
    }
    if (!w->mark || (numeric && (!w->acc || !w->absacc || !w->list))) {
        work_free(w);
        return -1;
    }
    for (int64_t j = 0; j < N; ++j) w->mark[j] = -1;
    return 0;
}

/* Symbolic step of the r-th listed row: its number of distinct columns. */
static void symbolic_row(const job_t *jb, work_t *w, int64_t r)
{
    int64_t i = jb->rows ? jb->rows[r] : r;
    int64_t count = 0;
    for (int64_t p = jb->arpt[i]; p < jb->arpt[i + 1]; ++p) {
        int64_t k = jb->acol[p];
        for (int64_t q = jb->brpt[k]; q < jb->brpt[k + 1]; ++q) {
            int32_t j = jb->bcol[q];
            if (w->mark[j] != r) {
                w->mark[j] = r;
                ++count;
            }
        }
    }
    jb->nnz[r] = count;
}

/* Numeric step of the r-th listed row into [off[r], off[r+1]).  Returns -2
 * when its size differs from the symbolic count. */
static int numeric_row(const job_t *jb, work_t *w, int64_t r)
{
    int64_t i = jb->rows ? jb->rows[r] : r;
    int64_t len = 0;
    for (int64_t p = jb->arpt[i]; p < jb->arpt[i + 1]; ++p) {
        int64_t k = jb->acol[p];
        double a = jb->aval[p];
        for (int64_t q = jb->brpt[k]; q < jb->brpt[k + 1]; ++q) {
            int32_t j = jb->bcol[q];
            double t = a * jb->bval[q];
            if (w->mark[j] != r) {
                w->mark[j] = r;
                w->acc[j] = t;
                w->absacc[j] = fabs(t);
                w->list[len++] = j;
            } else {
                w->acc[j] += t;
                w->absacc[j] += fabs(t);
            }
        }
    }
    if (len != jb->off[r + 1] - jb->off[r]) return -2;
    qsort(w->list, (size_t)len, sizeof(int32_t), cmp_i32);
    int64_t o = jb->off[r];
    for (int64_t e = 0; e < len; ++e) {
        int32_t j = w->list[e];
        jb->ccol[o + e] = j;
        jb->cval[o + e] = w->acc[j];
        if (jb->cabs) jb->cabs[o + e] = w->absacc[j];
    }
    return 0;
}

/* ---- several threads over blocks of rows ---------------------------------- */
#define ROW_BLOCK 64

typedef struct {
    const job_t *jb;
    int numeric;
    int64_t next;    /* next unclaimed block, atomically advanced */
    int rc;
} pool_t;

static void *pool_worker(void *arg)
{
    pool_t *pl = (pool_t *)arg;
    work_t w;
    if (work_init(&w, pl->jb->N, pl->numeric) != 0) {
        __atomic_store_n(&pl->rc, -1, __ATOMIC_RELAXED);
        return NULL;
    }
    for (;;) {
        int64_t b = __atomic_fetch_add(&pl->next, 1, __ATOMIC_RELAXED);
        int64_t r0 = b * ROW_BLOCK;
        if (r0 >= pl->jb->nr || __atomic_load_n(&pl->rc, __ATOMIC_RELAXED) != 0) break;
        int64_t r1 = r0 + ROW_BLOCK < pl->jb->nr ? r0 + ROW_BLOCK : pl->jb->nr;
        for (int64_t r = r0; r < r1; ++r) {
            if (pl->numeric) {
                int rc = numeric_row(pl->jb, &w, r);
                if (rc != 0) {
                    __atomic_store_n(&pl->rc, rc, __ATOMIC_RELAXED);
                    break;
                }
            } else {
                symbolic_row(pl->jb, &w, r);
            }
        }
    }
    work_free(&w);
    return NULL;
}

static int run_rows(const job_t *jb, int numeric, int nthreads)
{
    if (nthreads <= 1 || jb->nr <= ROW_BLOCK) {
        work_t w;
        if (work_init(&w, jb->N, numeric) != 0) return -1;
        int rc = 0;
        for (int64_t r = 0; r < jb->nr && rc == 0; ++r) {
            if (numeric) rc = numeric_row(jb, &w, r);
            else symbolic_row(jb, &w, r);
        }
        work_free(&w);
        return rc;
    }
    if (nthreads > 256) nthreads = 256;
    pool_t pl = {jb, numeric, 0, 0};
    pthread_t th[256];
    int started = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (pthread_create(&th[t], NULL, pool_worker, &pl) != 0) break;
        ++started;
    }
    if (started == 0) return run_rows(jb, numeric, 1);
    for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
    return pl.rc;
}

/* Symbolic: number of distinct output columns of each listed row.
 * rows == NULL means rows 0..nr-1.  nnz[r] receives the count of the r-th
 * listed row. */
int oracle_symbolic_mt(int nthreads, int64_t nr, const int64_t *rows, int64_t N,
                       const int64_t *arpt, const int32_t *acol,
                       const int64_t *brpt, const int32_t *bcol, int64_t *nnz)
{
    job_t jb;
    memset(&jb, 0, sizeof(jb));
    jb.nr = nr; jb.rows = rows; jb.N = N;
    jb.arpt = arpt; jb.acol = acol; jb.brpt = brpt; jb.bcol = bcol;
    jb.nnz = nnz;
    return run_rows(&jb, 0, nthreads);
}

int oracle_symbolic(int64_t nr, const int64_t *rows, int64_t N,
                    const int64_t *arpt, const int32_t *acol,
                    const int64_t *brpt, const int32_t *bcol, int64_t *nnz)
{
    return oracle_symbolic_mt(1, nr, rows, N, arpt, acol, brpt, bcol, nnz);
}

/* Numeric: fill each listed row r at offsets [off[r], off[r+1]) of
 * ccol/cval/cabs with its ascending columns, values and S scale.
 * off has nr+1 entries and must come from the symbolic counts. */
int oracle_numeric_mt(int nthreads, int64_t nr, const int64_t *rows, int64_t N,
                      const int64_t *arpt, const int32_t *acol, const double *aval,
                      const int64_t *brpt, const int32_t *bcol, const double *bval,
                      const int64_t *off, int32_t *ccol, double *cval, double *cabs)
{
    job_t jb;
    memset(&jb, 0, sizeof(jb));
    jb.nr = nr; jb.rows = rows; jb.N = N;
    jb.arpt = arpt; jb.acol = acol; jb.aval = aval;
    jb.brpt = brpt; jb.bcol = bcol; jb.bval = bval;
    jb.off = off; jb.ccol = ccol; jb.cval = cval; jb.cabs = cabs;
    return run_rows(&jb, 1, nthreads);
}

int oracle_numeric(int64_t nr, const int64_t *rows, int64_t N,
                   const int64_t *arpt, const int32_t *acol, const double *aval,
                   const int64_t *brpt, const int32_t *bcol, const double *bval,
                   const int64_t *off, int32_t *ccol, double *cval, double *cabs)
{
    return oracle_numeric_mt(1, nr, rows, N, arpt, acol, aval, brpt, bcol, bval, off,
                             ccol, cval, cabs);
}
