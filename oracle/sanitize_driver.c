/* Sanitizer driver for the CPU oracle (test infrastructure, never part of the GPU path).
 *
 * Built together with tsqr_oracle.c under AddressSanitizer and UndefinedBehaviorSanitizer
 * by tests/test_oracle_sanitize.py, it calls every exported oracle routine on small,
 * ragged inputs: leading dimensions above the row count, n = 1, s = n, odd sizes, a
 * zero column (breakdown) and a NaN entry, so that an out-of-bounds access, a use of
 * freed memory, a leak or undefined arithmetic in the oracle fails the CPU suite.
 * Exit status 0 when every call returned. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

double or_sketch_normal(uint64_t seed, int64_t i, int64_t j);
void or_sketch_normals(uint64_t seed, int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                       double *Zout, int64_t ldz);
void or_sketch_apply(int64_t m, int64_t n, const double *A, int64_t lda, int64_t s,
                     uint64_t seed, double *B, int64_t ldb);
void or_sample_rows(int64_t m, int64_t s, uint64_t seed, int64_t *rows);
void or_sketch_rows(int64_t m, int64_t n, const double *A, int64_t lda, int64_t s,
                    uint64_t seed, double *B, int64_t ldb);
int or_householder_r(int64_t s, int64_t n, const double *B, int64_t ldb, double *R,
                     int64_t ldr);
int or_lu_r(int64_t s, int64_t n, const double *B, int64_t ldb, double *R, int64_t ldr,
            int64_t *piv);
void or_trsm_ru(int64_t m, int64_t n, const double *Y, int64_t ldy, const double *T,
                int64_t ldt, double *X, int64_t ldx);
void or_gram(int64_t m, int64_t n, const double *X, int64_t ldx, double *W, int64_t ldw);
int or_cholesky_upper(int64_t n, const double *W, int64_t ldw, double *R, int64_t ldr);
void or_trmm_upper(int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
                   double *C, int64_t ldc);
int or_rxr_cholqr(int variant, int64_t m, int64_t n, const double *A, int64_t lda,
                  int64_t s, uint64_t seed, int extra_pass, double *Q, int64_t ldq,
                  double *R, int64_t ldr, double *R0o, double *R1o, double *R2o);
int or_rxr_cholqr_rows(int variant, int64_t m, int64_t n, const double *A, int64_t lda,
                       int64_t s, uint64_t seed, int extra_pass, double *Q, int64_t ldq,
                       double *R, int64_t ldr, double *R0o, double *R1o, double *R2o);
int or_lstsq_rxr(int variant, int sketch, int64_t m, int64_t n, const double *A, int64_t lda,
                 const double *b, int64_t s, uint64_t seed, double *x);
int or_cholqr_n(int64_t m, int64_t n, const double *A, int64_t lda, int npass,
                double shift, double *Q, int64_t ldq, double *R, int64_t ldr);
double or_orthogonality(int64_t m, int64_t n, const double *Q, int64_t ldq);
double or_residual(int64_t m, int64_t n, const double *A, int64_t lda, const double *Q,
                   int64_t ldq, const double *R, int64_t ldr);
double or_round_fp32(double x);
double or_round_bf16(double x);
void or_sketch_apply_lowp(int prec, int64_t m, int64_t n, const double *A, int64_t lda,
                          int64_t s, uint64_t seed, double *B, int64_t ldb);
void or_apply_rinv_lowp(int prec, int64_t m, int64_t n, const double *Y, int64_t ldy,
                        const double *Rinv, int64_t ldr, double *X, int64_t ldx);
void or_gram_lowp(int prec, int64_t m, int64_t n, const double *X, int64_t ldx, double *W,
                  int64_t ldw);
void or_trtri_upper(int64_t n, const double *T, int64_t ldt, double *X, int64_t ldx);
int or_rxr_cholqr_mixed(int variant, int prec, int64_t m, int64_t n, const double *A,
                        int64_t lda, int64_t s, uint64_t seed, int fp64_passes, double *Q,
                        int64_t ldq, double *R, int64_t ldr, int *lp_info, int *passes_out);

/* A full-rank m x n matrix (leading dimension lda) of smooth, distinct columns plus a
 * scaled diagonal; exact values do not matter here. */
static double *make(int64_t m, int64_t n, int64_t lda) {
    double *A = (double *)malloc((size_t)lda * (size_t)n * sizeof(double));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < lda; ++i)
            A[i + j * lda] = (i < m) ? sin(0.37 * (double)(i + 1) * (double)(j + 1) + 0.1 * j) +
                                           (i == j ? 2.0 : 0.0)
                                     : -12345.0; /* padding rows, never read as data */
    return A;
}

static void run_shape(int64_t m, int64_t n, int64_t s, int64_t pad) {
    const int64_t lda = m + pad, ldq = m + pad, ldr = n + pad;
    double *A = make(m, n, lda);
    double *Q = (double *)malloc((size_t)ldq * (size_t)n * sizeof(double));
    double *R = (double *)malloc((size_t)ldr * (size_t)n * sizeof(double));
    double *R0 = (double *)malloc((size_t)n * (size_t)n * sizeof(double));
    double *R1 = (double *)malloc((size_t)n * (size_t)n * sizeof(double));
    double *R2 = (double *)malloc((size_t)n * (size_t)n * sizeof(double));
    double *B = (double *)malloc((size_t)(s + pad) * (size_t)n * sizeof(double));
    double *Z = (double *)malloc((size_t)s * (size_t)m * sizeof(double));
    double *W = (double *)malloc((size_t)ldr * (size_t)n * sizeof(double));
    double *X = (double *)malloc((size_t)ldq * (size_t)n * sizeof(double));
    double *b = (double *)malloc((size_t)m * sizeof(double));
    double *x = (double *)malloc((size_t)n * sizeof(double));
    int64_t *piv = (int64_t *)malloc((size_t)s * sizeof(int64_t));
    int64_t *rows = (int64_t *)malloc((size_t)s * sizeof(int64_t));
    for (int64_t i = 0; i < m; ++i) b[i] = cos(0.1 * (double)i);

    (void)or_sketch_normal(7, 3, m - 1);
    or_sketch_normals(7, 0, s, 0, m, Z, s);
    or_sketch_apply(m, n, A, lda, s, 7, B, s + pad);
    or_sample_rows(m, s, 7, rows);
    or_sketch_rows(m, n, A, lda, s, 7, B, s + pad);
    (void)or_householder_r(s, n, B, s + pad, R, ldr);
    (void)or_lu_r(s, n, B, s + pad, R, ldr, piv);
    or_trsm_ru(m, n, A, lda, R, ldr, X, ldq);
    or_gram(m, n, X, ldq, W, ldr);
    (void)or_cholesky_upper(n, W, ldr, R1, n);
    or_trmm_upper(n, R1, n, R, ldr, R2, n);
    for (int variant = 0; variant < 2; ++variant)
        for (int extra = 0; extra < 2; ++extra) {
            (void)or_rxr_cholqr(variant, m, n, A, lda, s, 9, extra, Q, ldq, R, ldr, R0, R1, R2);
            (void)or_rxr_cholqr(variant, m, n, A, lda, s, 9, extra, Q, ldq, R, ldr, NULL, NULL,
                                NULL);
            (void)or_rxr_cholqr_rows(variant, m, n, A, lda, s, 9, extra, Q, ldq, R, ldr, R0,
                                     R1, R2);
            (void)or_lstsq_rxr(variant, extra, m, n, A, lda, b, s, 9, x);
        }
    for (int npass = 1; npass <= 3; ++npass) {
        (void)or_cholqr_n(m, n, A, lda, npass, 0.0, Q, ldq, R, ldr);
        (void)or_cholqr_n(m, n, A, lda, npass, -1.0, Q, ldq, R, ldr);
    }
    (void)or_orthogonality(m, n, Q, ldq);
    (void)or_residual(m, n, A, lda, Q, ldq, R, ldr);
    (void)or_round_fp32(1.0 / 3.0);
    (void)or_round_bf16(1.0 / 3.0);
    for (int prec = 1; prec <= 2; ++prec) {
        int lp = 0, passes = 0;
        or_sketch_apply_lowp(prec, m, n, A, lda, s, 7, B, s + pad);
        or_trtri_upper(n, R1, n, R0, n);
        or_apply_rinv_lowp(prec, m, n, A, lda, R0, n, X, ldq);
        or_gram_lowp(prec, m, n, X, ldq, W, ldr);
        for (int fp = 0; fp <= 3; ++fp)
            (void)or_rxr_cholqr_mixed(1 - (prec & 1), prec, m, n, A, lda, s, 9, fp, Q, ldq, R,
                                      ldr, &lp, &passes);
    }
    /* breakdowns: a zero column, then a NaN entry */
    for (int64_t i = 0; i < m; ++i) A[i + (n / 2) * lda] = 0.0;
    (void)or_rxr_cholqr(0, m, n, A, lda, s, 9, 1, Q, ldq, R, ldr, R0, R1, R2);
    (void)or_rxr_cholqr(1, m, n, A, lda, s, 9, 1, Q, ldq, R, ldr, R0, R1, R2);
    (void)or_cholqr_n(m, n, A, lda, 2, 0.0, Q, ldq, R, ldr);
    A[m / 3] = NAN;
    (void)or_rxr_cholqr(0, m, n, A, lda, s, 9, 1, Q, ldq, R, ldr, R0, R1, R2);
    (void)or_lstsq_rxr(0, 0, m, n, A, lda, b, s, 9, x);
    {
        int lp = 0, passes = 0;
        (void)or_rxr_cholqr_mixed(0, 2, m, n, A, lda, s, 9, 0, Q, ldq, R, ldr, &lp, &passes);
    }
    free(A); free(Q); free(R); free(R0); free(R1); free(R2); free(B); free(Z); free(W);
    free(X); free(b); free(x); free(piv); free(rows);
}

int main(void) {
    const int64_t shapes[][4] = {{257, 1, 1, 3}, {300, 7, 7, 0}, {513, 17, 35, 5},
                                 {1000, 40, 80, 1}, {130, 65, 129, 2}};
    for (size_t k = 0; k < sizeof shapes / sizeof shapes[0]; ++k) {
        run_shape(shapes[k][0], shapes[k][1], shapes[k][2], shapes[k][3]);
        printf("shape m=%lld n=%lld s=%lld pad=%lld done\n", (long long)shapes[k][0],
               (long long)shapes[k][1], (long long)shapes[k][2], (long long)shapes[k][3]);
    }
    return 0;
}
