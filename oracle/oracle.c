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
 * Method: single thread, dense accumulator indexed by column with a
 * "last row that touched this column" marker, plus the list of touched
 * columns, sorted at the end of the row with the C library's qsort.
 * Products are summed in ascending k (A rows are sorted), then in B-row order,
 * each product rounded to double before the add (build with
 * -ffp-contract=off so no fused multiply-add merges the two roundings).
 * Alongside each value it accumulates S_ij = sum_k |A_ik * B_kj|, the scale
 * that bounds the rounding error of any summation order.
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

/* Symbolic: number of distinct output columns of each listed row.
 * rows == NULL means rows 0..nr-1.  nnz[r] receives the count of the r-th
 * listed row. */
int oracle_symbolic(int64_t nr, const int64_t *rows, int64_t N,
                    const int64_t *arpt, const int32_t *acol,
                    const int64_t *brpt, const int32_t *bcol, int64_t *nnz)
{
    int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    if (!mark) return -1;
    for (int64_t j = 0; j < N; ++j) mark[j] = -1;
    for (int64_t r = 0; r < nr; ++r) {
        int64_t i = rows ? rows[r] : r;
        int64_t count = 0;
        for (int64_t p = arpt[i]; p < arpt[i + 1]; ++p) {
            int64_t k = acol[p];
            for (int64_t q = brpt[k]; q < brpt[k + 1]; ++q) {
                int32_t j = bcol[q];
                if (mark[j] != r) {
                    mark[j] = r;
                    ++count;
                }
            }
        }
        nnz[r] = count;
    }
    free(mark);
    return 0;
}

/* Numeric: fill each listed row r at offsets [off[r], off[r+1]) of
 * ccol/cval/cabs with its ascending columns, values and S scale.
 * off has nr+1 entries and must come from the symbolic counts. */
int oracle_numeric(int64_t nr, const int64_t *rows, int64_t N,
                   const int64_t *arpt, const int32_t *acol, const double *aval,
                   const int64_t *brpt, const int32_t *bcol, const double *bval,
                   const int64_t *off, int32_t *ccol, double *cval, double *cabs)
{
    size_t n = (size_t)(N > 0 ? N : 1);
    int64_t *mark = (int64_t *)malloc(sizeof(int64_t) * n);
    double *acc = (double *)malloc(sizeof(double) * n);
    double *absacc = (double *)malloc(sizeof(double) * n);
    int32_t *list = (int32_t *)malloc(sizeof(int32_t) * n);
    if (!mark || !acc || !absacc || !list) {
        free(mark); free(acc); free(absacc); free(list);
        return -1;
    }
    for (int64_t j = 0; j < N; ++j) mark[j] = -1;
    int rc = 0;
    for (int64_t r = 0; r < nr; ++r) {
        int64_t i = rows ? rows[r] : r;
        int64_t len = 0;
        for (int64_t p = arpt[i]; p < arpt[i + 1]; ++p) {
            int64_t k = acol[p];
            double a = aval[p];
            for (int64_t q = brpt[k]; q < brpt[k + 1]; ++q) {
                int32_t j = bcol[q];
                double t = a * bval[q];
                if (mark[j] != r) {
                    mark[j] = r;
                    acc[j] = t;
                    absacc[j] = fabs(t);
                    list[len++] = j;
                } else {
                    acc[j] += t;
                    absacc[j] += fabs(t);
                }
            }
        }
        if (len != off[r + 1] - off[r]) { rc = -2; break; }
        qsort(list, (size_t)len, sizeof(int32_t), cmp_i32);
        int64_t o = off[r];
        for (int64_t e = 0; e < len; ++e) {
            int32_t j = list[e];
            ccol[o + e] = j;
            cval[o + e] = acc[j];
            if (cabs) cabs[o + e] = absacc[j];
        }
    }
    free(mark); free(acc); free(absacc); free(list);
    return rc;
}
