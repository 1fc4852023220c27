/*
 * ORACLE (test infrastructure only).  Plain FP64 CSR sparse x dense product.
 *
 * The arrow decomposition is an exact rewriting of A (Section 4, Eq. (1):
 * A X = sum_i P_i (B_i (P_i^T X)), and every nonzero of A lands in exactly one
 * B_i, Section 6.2 storage lemma).  The method therefore reaches Y = A X up to
 * rounding order, and this file is that plain definition written out:
 *
 *     Y[i, :] = sum over stored entries p of row i of  val[p] * X[col[p], :]
 *
 * summed in stored (ascending column) order, in double precision.  Rows are
 * independent; OpenMP only splits the row loop across threads and does not
 * change the order of any sum.
 *
 * Nothing here is shared with the HIP path.
 */
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the row loops below (timing of the oracle on fewer cores). */
void oracle_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Y (n x k, row-major, ld k) = A (CSR, n x n) * X (n x k, row-major, ld k). */
void oracle_csr_spmm_f64(int64_t n, const int64_t *row_ptr, const int32_t *col,
                         const float *val, const double *X, int64_t k, double *Y) {
    int64_t i;
#pragma omp parallel for schedule(dynamic, 1024)
    for (i = 0; i < n; ++i) {
        double *y = Y + i * k;
        for (int64_t j = 0; j < k; ++j) y[j] = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            const double a = (double)val[p];
            const double *x = X + (int64_t)col[p] * k;
            for (int64_t j = 0; j < k; ++j) y[j] += a * x[j];
        }
    }
}

/* Same product for a subset of rows: Y[r, :] = (A X)[rows[r], :]. X is only
 * read at the columns those rows touch, so X may be a full n x k matrix while
 * Y has nrows x k entries. */
void oracle_csr_spmm_rows_f64(const int64_t *row_ptr, const int32_t *col, const float *val,
                              const double *X, int64_t k, const int64_t *rows,
                              int64_t nrows, double *Y) {
    int64_t r;
#pragma omp parallel for schedule(dynamic, 64)
    for (r = 0; r < nrows; ++r) {
        const int64_t i = rows[r];
        double *y = Y + r * k;
        for (int64_t j = 0; j < k; ++j) y[j] = 0.0;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            const double a = (double)val[p];
            const double *x = X + (int64_t)col[p] * k;
            for (int64_t j = 0; j < k; ++j) y[j] += a * x[j];
        }
    }
}

/* Column sums of squares of an n x k row-major matrix, accumulated row by
 * row in index order (a sequential sum per column). */
void oracle_col_sumsq_f64(int64_t n, int64_t k, const double *Y, double *out) {
    for (int64_t j = 0; j < k; ++j) out[j] = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < k; ++j) out[j] += Y[i * k + j] * Y[i * k + j];
}
