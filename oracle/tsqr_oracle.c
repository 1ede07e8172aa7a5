/*
 * tsqr_oracle.c -- slow, plain FP64 CPU reference of randomized XR-preconditioned
 * CholeskyQR (Fan, Guo, Lin, "A Novel Randomized XR-Based Preconditioned CholeskyQR
 * Algorithm", arXiv 2111.11148).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the package entry
 * point and the CPU-baseline leg of the benchmark may load this library.  The GPU library
 * never links, includes or calls anything here, and nothing here calls the GPU library.
 *
 * Conventions
 *   - every matrix is column-major with an explicit leading dimension (LAPACK style);
 *     element (i, j) of X lives at X[i + j*ldx];
 *   - arithmetic is IEEE binary64, compiled with -ffp-contract=off so each line below is
 *     exactly the rounding sequence it reads as (no fused multiply-add unless written);
 *   - loops are the plain definitions; OpenMP only splits loops over independent outputs
 *     (rows of a solve, entries of a product), never the order of a sum;
 *   - `info` codes: 0 = success; 1000*stage + k = non-positive, zero or NaN pivot at the
 *     k-th (1-based) column of stage `stage` (1 = sketch factor R0, 2 = first Cholesky
 *     R1, 3 = second Cholesky R2, 4 = any further Cholesky pass).  On breakdown the
 *     outputs Q and R are filled with NaN.
 *
 * Pins: the paper prints no worked numerical example (its accuracy and runtime figures
 * are absent from the text), so no function here is checked against a value the paper
 * prints; each is pinned instead by closed forms, invariants, brute force, independent
 * library implementations (NumPy's Philox, LAPACK, torch's BF16 rounding, mpmath) and the
 * bounds the paper states (see tests/test_oracle_pins.py, tests/test_oracle_mixed_pins.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

static double or_fro(int64_t n, const double *X, int64_t ldx);

/* ------------------------------------------------------------------------------------
 * Counter-based generator: Philox-4xW-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11).  One round maps the counter (c0,c1,c2,c3) with
 * key (k0,k1) to
 *     (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0));
 * between rounds the key is bumped by the Weyl constants (W0, W1).  Ten rounds.
 * The same round is written once and instantiated for 32- and 64-bit words, so that the
 * 64-bit instance (cross-checked against an independent implementation) also vouches
 * for the round structure of the 32-bit instance the sketch uses.
 * ------------------------------------------------------------------------------------ */
static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

static inline void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

#define PHILOX_4xW_10(NAME, T, MULHILO, M0, M1, W0, W1)                                  \
    void NAME(const T ctr[4], const T key[2], T out[4]) {                                \
        T c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];                            \
        T k0 = key[0], k1 = key[1];                                                      \
        for (int round = 0; round < 10; ++round) {                                       \
            if (round > 0) {                                                             \
                k0 = (T)(k0 + (W0));                                                     \
                k1 = (T)(k1 + (W1));                                                     \
            }                                                                            \
            T hi0, lo0, hi1, lo1;                                                        \
            MULHILO((M0), c0, &hi0, &lo0);                                               \
            MULHILO((M1), c2, &hi1, &lo1);                                               \
            T n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;                \
            c0 = n0; c1 = n1; c2 = n2; c3 = n3;                                          \
        }                                                                                \
        out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;                              \
    }

PHILOX_4xW_10(or_philox4x32_10, uint32_t, mulhilo32, 0xD2511F53u, 0xCD9E8D57u,
              0x9E3779B9u, 0xBB67AE85u)
PHILOX_4xW_10(or_philox4x64_10, uint64_t, mulhilo64, 0xD2E7470EE14C6C93ull,
              0xCA5A826395121157ull, 0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull)

/* ------------------------------------------------------------------------------------
 * The Gaussian sketch (paper Section 2.3, "Gaussian Ensemble": A1 = Omega*A with i.i.d.
 * standard normal Omega).  The sketch used here is S = Z / sqrt(s), Z(i,j) ~ N(0,1).
 *
 * Stream layout (a reading; the paper does not fix a generator):
 *   key = (low 32 bits of seed, high 32 bits of seed)
 *   one Philox4x32-10 call yields the four entries Z(i, 4p .. 4p+3) of row i, with
 *   counter = (low 32 bits of p, high 32 bits of p, i, 0);
 *   words (w0,w1) give columns 4p, 4p+1 and (w2,w3) columns 4p+2, 4p+3 by Box-Muller
 *   (Box & Muller 1958) on 24-bit uniforms:
 *       u = ((w_a >> 8) + 1) * 2^-24  in (0, 1],   t = (w_b >> 8) * 2^-24  in [0, 1),
 *       rad = sqrt(-2 ln u),  first of the pair = rad*cos(2 pi t), second = rad*sin(2 pi t).
 * ------------------------------------------------------------------------------------ */
double or_sketch_normal(uint64_t seed, int64_t i, int64_t j) {
    uint64_t p = (uint64_t)j >> 2;
    int col = (int)(j & 3);
    uint32_t ctr[4] = {(uint32_t)p, (uint32_t)(p >> 32), (uint32_t)i, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    uint32_t wa = w[(col >> 1) * 2], wb = w[(col >> 1) * 2 + 1];
    double u = ((double)(wa >> 8) + 1.0) * 0x1p-24;
    double t = (double)(wb >> 8) * 0x1p-24;
    double rad = sqrt(-2.0 * log(u));
    double ang = 2.0 * M_PI * t;
    return (col & 1) ? rad * sin(ang) : rad * cos(ang);
}

/* Z(i0+a, j0+b) for a < ni, b < nj into Zout (ld ldz).  Debug / test helper. */
void or_sketch_normals(uint64_t seed, int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                       double *Zout, int64_t ldz) {
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nj; ++b)
        for (int64_t a = 0; a < ni; ++a)
            Zout[IDX(a, b, ldz)] = or_sketch_normal(seed, i0 + a, j0 + b);
}

/* Sketch: B = S*A with S(i,j) = Z(i,j)/sqrt(s); B is s x n (paper Section 2.3).  Each
 * entry is the plain sum over j = 0..m-1 in increasing order. */
void or_sketch_apply(int64_t m, int64_t n, const double *A, int64_t lda, int64_t s,
                     uint64_t seed, double *B, int64_t ldb) {
    double rs = 1.0 / sqrt((double)s);
#pragma omp parallel
    {
        double *srow = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < s; ++i) {
            for (int64_t j = 0; j < m; ++j) srow[j] = or_sketch_normal(seed, i, j) * rs;
            for (int64_t c = 0; c < n; ++c) {
                double acc = 0.0;
                const double *acol = A + IDX(0, c, lda);
                for (int64_t j = 0; j < m; ++j) acc += srow[j] * acol[j];
                B[IDX(i, c, ldb)] = acc;
            }
        }
        free(srow);
    }
}

/* ------------------------------------------------------------------------------------
 * The row-extraction sketch (paper Section 2.3, "Row Extraction", the sketch of its
 * experiments), with the sampling of Theorem "Equal Probability Case": s rows drawn
 * independently, each uniformly from the m rows, so a row may repeat.  B(i, :) = A(r_i, :)
 * (P selects rows, no scaling).
 *
 * Stream layout (a reading; the paper does not fix a generator): key as for the Gaussian
 * sketch; for draw i, one Philox4x32-10 call with counter = (low 32 bits of i, high 32
 * bits of i, 0, 1) (the last word is 0 for every Gaussian-sketch counter, so the streams
 * never meet); w = w0 + 2^32 w1 and r_i = floor(w m / 2^64), exact 128-bit arithmetic.
 * ------------------------------------------------------------------------------------ */
void or_sample_rows(int64_t m, int64_t s, uint64_t seed, int64_t *rows) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < s; ++i) {
        uint32_t ctr[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), 0u, 1u};
        uint32_t w[4];
        or_philox4x32_10(ctr, key, w);
        uint64_t w64 = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
        rows[i] = (int64_t)(((unsigned __int128)w64 * (unsigned __int128)(uint64_t)m) >> 64);
    }
}

void or_sketch_rows(int64_t m, int64_t n, const double *A, int64_t lda, int64_t s,
                    uint64_t seed, double *B, int64_t ldb) {
    int64_t *rows = (int64_t *)malloc((size_t)s * sizeof(int64_t));
    or_sample_rows(m, s, seed, rows);
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < s; ++i) B[IDX(i, j, ldb)] = A[IDX(rows[i], j, lda)];
    free(rows);
}

/* ------------------------------------------------------------------------------------
 * Small dense factorizations of the l x n sketch (the R factor of the sketch in paper
 * Algorithms rLU- and rQR-CholeskyQR).
 * ------------------------------------------------------------------------------------ */

/* Householder QR (Golub & Van Loan, "Matrix Computations", Alg. 5.2.1 with the reflector
 * of Alg. 5.1.1 in LAPACK's sign convention: beta = -sign(alpha)*||x||, sign(0) = +1).
 * Only R is kept (Q-less QR, paper footnote to the rQR algorithm).  The result is then
 * sign-normalised, R0 = diag(sign r_kk) * R, so that its diagonal is positive.
 * R (n x n, ld ldr) gets the upper triangle; its strict lower triangle is zeroed.
 * Returns 0, or 1000 + k when column k (1-based) has a zero or NaN diagonal. */
int or_householder_r(int64_t s, int64_t n, const double *B, int64_t ldb, double *R,
                     int64_t ldr) {
    double *W = (double *)malloc((size_t)s * (size_t)n * sizeof(double));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < s; ++i) W[IDX(i, j, s)] = B[IDX(i, j, ldb)];
    double *v = (double *)malloc((size_t)s * sizeof(double));
    int info = 0;
    for (int64_t k = 0; k < n && k < s; ++k) {
        double alpha = W[IDX(k, k, s)];
        double xnorm2 = 0.0;
        for (int64_t i = k + 1; i < s; ++i) xnorm2 += W[IDX(i, k, s)] * W[IDX(i, k, s)];
        double tau;
        if (xnorm2 == 0.0) {
            /* nothing below the diagonal: identity reflector */
            tau = 0.0;
            v[k] = 1.0;
            for (int64_t i = k + 1; i < s; ++i) v[i] = 0.0;
        } else {
            double norm = sqrt(alpha * alpha + xnorm2);
            double beta = (alpha >= 0.0) ? -norm : norm;
            tau = (beta - alpha) / beta;
            double scal = 1.0 / (alpha - beta);
            v[k] = 1.0;
            for (int64_t i = k + 1; i < s; ++i) v[i] = W[IDX(i, k, s)] * scal;
            W[IDX(k, k, s)] = beta;
            for (int64_t i = k + 1; i < s; ++i) W[IDX(i, k, s)] = 0.0;
        }
        /* apply H = I - tau v v^T to the trailing columns */
        for (int64_t j = k + 1; j < n; ++j) {
            double w = 0.0;
            for (int64_t i = k; i < s; ++i) w += v[i] * W[IDX(i, j, s)];
            w *= tau;
            for (int64_t i = k; i < s; ++i) W[IDX(i, j, s)] -= v[i] * w;
        }
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) R[IDX(i, j, ldr)] = (i <= j && i < s) ? W[IDX(i, j, s)] : 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double d = R[IDX(k, k, ldr)];
        if (!(d != 0.0) || isnan(d)) {
            if (!info) info = 1000 + (int)(k + 1);
            continue;
        }
        if (d < 0.0)
            for (int64_t j = k; j < n; ++j) R[IDX(k, j, ldr)] = -R[IDX(k, j, ldr)];
    }
    free(v);
    free(W);
    return info;
}

/* Gaussian elimination with partial (row) pivoting (Golub & Van Loan, Alg. 3.4.1): the
 * pivot of column k is the first row index of the largest |b_ik|, i >= k.  Only U is
 * kept, then R0 = diag(sign u_kk) * U.  piv (optional, length n) receives the 0-based
 * row chosen at each step.  Returns 0 or 1000 + k for a zero or NaN pivot. */
int or_lu_r(int64_t s, int64_t n, const double *B, int64_t ldb, double *R, int64_t ldr,
            int64_t *piv) {
    double *W = (double *)malloc((size_t)s * (size_t)n * sizeof(double));
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < s; ++i) W[IDX(i, j, s)] = B[IDX(i, j, ldb)];
    int info = 0;
    for (int64_t k = 0; k < n && k < s; ++k) {
        int64_t p = k;
        double best = fabs(W[IDX(k, k, s)]);
        for (int64_t i = k + 1; i < s; ++i) {
            double a = fabs(W[IDX(i, k, s)]);
            if (a > best) { best = a; p = i; }
        }
        if (piv) piv[k] = p;
        if (p != k)
            for (int64_t j = 0; j < n; ++j) {
                double t = W[IDX(k, j, s)];
                W[IDX(k, j, s)] = W[IDX(p, j, s)];
                W[IDX(p, j, s)] = t;
            }
        double pv = W[IDX(k, k, s)];
        if (!(pv != 0.0) || isnan(pv)) {
            if (!info) info = 1000 + (int)(k + 1);
            continue;
        }
        for (int64_t i = k + 1; i < s; ++i) W[IDX(i, k, s)] /= pv;
        for (int64_t j = k + 1; j < n; ++j)
            for (int64_t i = k + 1; i < s; ++i)
                W[IDX(i, j, s)] -= W[IDX(i, k, s)] * W[IDX(k, j, s)];
    }
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) R[IDX(i, j, ldr)] = (i <= j && i < s) ? W[IDX(i, j, s)] : 0.0;
    if (!info)
        for (int64_t k = 0; k < n; ++k)
            if (R[IDX(k, k, ldr)] < 0.0)
                for (int64_t j = k; j < n; ++j) R[IDX(k, j, ldr)] = -R[IDX(k, j, ldr)];
    free(W);
    return info;
}

/* ------------------------------------------------------------------------------------
 * Tall-skinny kernels of CholeskyQR (paper Algorithm CholeskyQR).
 * ------------------------------------------------------------------------------------ */

/* X = Y * T^{-1}, T upper triangular n x n: row-by-row forward substitution,
 *   x_j = (y_j - sum_{k<j} x_k t_kj) / t_jj   (sum in increasing k).
 * X may alias Y (same pointer and leading dimension). */
void or_trsm_ru(int64_t m, int64_t n, const double *Y, int64_t ldy, const double *T,
                int64_t ldt, double *X, int64_t ldx) {
#pragma omp parallel
    {
        double *x = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t j = 0; j < n; ++j) {
                double acc = Y[IDX(i, j, ldy)];
                for (int64_t k = 0; k < j; ++k) acc -= x[k] * T[IDX(k, j, ldt)];
                x[j] = acc / T[IDX(j, j, ldt)];
            }
            for (int64_t j = 0; j < n; ++j) X[IDX(i, j, ldx)] = x[j];
        }
        free(x);
    }
}

/* Gram matrix W = X^T X (the Gram matrix of paper Algorithm CholeskyQR).  Only the upper triangle
 * (with the diagonal) is formed; the strict lower triangle of W is set equal to it. */
void or_gram(int64_t m, int64_t n, const double *X, int64_t ldx, double *W, int64_t ldw) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < n; ++b)
        for (int64_t a = 0; a <= b; ++a) {
            const double *xa = X + IDX(0, a, ldx), *xb = X + IDX(0, b, ldx);
            double acc = 0.0;
            for (int64_t j = 0; j < m; ++j) acc += xa[j] * xb[j];
            W[IDX(a, b, ldw)] = acc;
            W[IDX(b, a, ldw)] = acc;
        }
}

/* Cholesky W = R^T R, R upper (Golub & Van Loan, Alg. 4.2.1 in its row-oriented form):
 *   r_kk = sqrt(w_kk - sum_{i<k} r_ik^2),  r_kj = (w_kj - sum_{i<k} r_ik r_ij) / r_kk.
 * Reads the upper triangle of W.  Returns 0, or k (1-based) at the first pivot argument
 * that is not positive (or is NaN); R is then NaN from that column on. */
int or_cholesky_upper(int64_t n, const double *W, int64_t ldw, double *R, int64_t ldr) {
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) R[IDX(i, j, ldr)] = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double d = W[IDX(k, k, ldw)];
        for (int64_t i = 0; i < k; ++i) d -= R[IDX(i, k, ldr)] * R[IDX(i, k, ldr)];
        if (!(d > 0.0)) {
            for (int64_t j = k; j < n; ++j)
                for (int64_t i = 0; i <= j; ++i) R[IDX(i, j, ldr)] = NAN;
            return (int)(k + 1);
        }
        double rkk = sqrt(d);
        R[IDX(k, k, ldr)] = rkk;
        for (int64_t j = k + 1; j < n; ++j) {
            double a = W[IDX(k, j, ldw)];
            for (int64_t i = 0; i < k; ++i) a -= R[IDX(i, k, ldr)] * R[IDX(i, j, ldr)];
            R[IDX(k, j, ldr)] = a / rkk;
        }
    }
    return 0;
}

/* C = A * B for upper-triangular n x n A, B (C upper, strict lower zeroed):
 *   c_ij = sum_{i<=k<=j} a_ik b_kj.  C must not alias A or B. */
void or_trmm_upper(int64_t n, const double *A, int64_t lda, const double *B, int64_t ldb,
                   double *C, int64_t ldc) {
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) {
            double acc = 0.0;
            if (i <= j)
                for (int64_t k = i; k <= j; ++k) acc += A[IDX(i, k, lda)] * B[IDX(k, j, ldb)];
            C[IDX(i, j, ldc)] = acc;
        }
}

static void fill_nan(int64_t rows, int64_t cols, double *X, int64_t ldx) {
    if (!X) return;
    for (int64_t j = 0; j < cols; ++j)
        for (int64_t i = 0; i < rows; ++i) X[IDX(i, j, ldx)] = NAN;
}

/* One CholeskyQR pass (paper Algorithm CholeskyQR): W = X^T X, R = chol(W),
 * Xout = X R^{-1}.  Xout may alias X.  Returns the Cholesky info (0 or column). */
static int cholqr_pass(int64_t m, int64_t n, const double *X, int64_t ldx, double *Xout,
                       int64_t ldo, double *R, int64_t ldr) {
    double *W = (double *)malloc((size_t)n * (size_t)n * sizeof(double));
    or_gram(m, n, X, ldx, W, n);
    int info = or_cholesky_upper(n, W, n, R, ldr);
    free(W);
    if (info) return info;
    or_trsm_ru(m, n, X, ldx, R, ldr, Xout, ldo);
    return 0;
}

/* ------------------------------------------------------------------------------------
 * Drivers.
 * ------------------------------------------------------------------------------------ */

/* Randomized XR-preconditioned CholeskyQR (paper Algorithms rLU-CholeskyQR and
 * rQR-CholeskyQR, with the Gaussian sketch of Section 2.3), optionally followed by one
 * more CholeskyQR pass (paper Algorithm CholeskyQR2, second line):
 *   B  = S A                      (s x n)
 *   R0 = R factor of B            (variant 0: Householder QR; 1: partial-pivot LU)
 *   A1 = A R0^{-1}
 *   R1 = chol(A1^T A1),  Q1 = A1 R1^{-1}
 *   extra pass: R2 = chol(Q1^T Q1), Q = Q1 R2^{-1}, R = R2 (R1 R0);  else Q = Q1, R = R1 R0
 * Q is m x n (ld ldq), R is n x n upper (ld ldr).  R0, R1, R2 (n x n, ld n) are written
 * when the pointers are non-NULL (R2 only with the extra pass). */
static int rxr_cholqr_k(int sketch, int variant, int64_t m, int64_t n, const double *A,
                        int64_t lda, int64_t s, uint64_t seed, int extra_pass, double *Q,
                        int64_t ldq, double *R, int64_t ldr, double *R0o, double *R1o,
                        double *R2o) {
    size_t nn = (size_t)n * (size_t)n;
    double *B = (double *)malloc((size_t)s * (size_t)n * sizeof(double));
    double *R0 = (double *)calloc(nn, sizeof(double));
    double *R1 = (double *)calloc(nn, sizeof(double));
    double *R2 = (double *)calloc(nn, sizeof(double));
    double *R10 = (double *)calloc(nn, sizeof(double));
    int info = 0;

    if (sketch == 1) or_sketch_rows(m, n, A, lda, s, seed, B, s);
    else or_sketch_apply(m, n, A, lda, s, seed, B, s);
    info = (variant == 1) ? or_lu_r(s, n, B, s, R0, n, NULL) : or_householder_r(s, n, B, s, R0, n);
    if (!info) {
        or_trsm_ru(m, n, A, lda, R0, n, Q, ldq); /* Q holds A1 */
        int c = cholqr_pass(m, n, Q, ldq, Q, ldq, R1, n);
        if (c) info = 2000 + c;
    }
    if (!info) {
        or_trmm_upper(n, R1, n, R0, n, R10, n);
        if (extra_pass) {
            int c = cholqr_pass(m, n, Q, ldq, Q, ldq, R2, n);
            if (c) info = 3000 + c;
            else or_trmm_upper(n, R2, n, R10, n, R, ldr);
        } else {
            for (int64_t j = 0; j < n; ++j)
                for (int64_t i = 0; i < n; ++i) R[IDX(i, j, ldr)] = R10[IDX(i, j, n)];
        }
    }
    if (info) {
        fill_nan(m, n, Q, ldq);
        fill_nan(n, n, R, ldr);
    }
    if (R0o) memcpy(R0o, R0, nn * sizeof(double));
    if (R1o) memcpy(R1o, R1, nn * sizeof(double));
    if (R2o) memcpy(R2o, R2, nn * sizeof(double));
    free(B); free(R0); free(R1); free(R2); free(R10);
    return info;
}

int or_rxr_cholqr(int variant, int64_t m, int64_t n, const double *A, int64_t lda,
                  int64_t s, uint64_t seed, int extra_pass, double *Q, int64_t ldq,
                  double *R, int64_t ldr, double *R0o, double *R1o, double *R2o) {
    return rxr_cholqr_k(0, variant, m, n, A, lda, s, seed, extra_pass, Q, ldq, R, ldr, R0o,
                        R1o, R2o);
}

/* The same method with the row-extraction sketch in place of the Gaussian one. */
int or_rxr_cholqr_rows(int variant, int64_t m, int64_t n, const double *A, int64_t lda,
                       int64_t s, uint64_t seed, int extra_pass, double *Q, int64_t ldq,
                       double *R, int64_t ldr, double *R0o, double *R1o, double *R2o) {
    return rxr_cholqr_k(1, variant, m, n, A, lda, s, seed, extra_pass, Q, ldq, R, ldr, R0o,
                        R1o, R2o);
}

/* ------------------------------------------------------------------------------------
 * Least squares min ||A x - b||_2 preconditioned by the sketch's R factor (paper Section
 * 5.2, Algorithm "LS solver preconditioned by randomized R factor"; the paper's R_1 is
 * the R0 of the methods above):
 *   R0 = R factor of the sketch (Gaussian: sketch = 0, row extraction: sketch = 1; QR or
 *        LU by variant);
 *   B = A R0^{-1};
 *   y = (B^T B)^{-1} B^T b, by the normal equation: G = B^T B = U^T U (Cholesky),
 *       c = B^T b, U^T z = c, U y = z;
 *   x = R0^{-1} y  (R0 x = y).
 * Returns 0, or 1000 + k (small factorization), 2000 + k (Cholesky of G); x NaN then.
 * ------------------------------------------------------------------------------------ */
int or_lstsq_rxr(int variant, int sketch, int64_t m, int64_t n, const double *A, int64_t lda,
                 const double *b, int64_t s, uint64_t seed, double *x) {
    size_t nn = (size_t)n * (size_t)n;
    double *Bs = (double *)malloc((size_t)s * (size_t)n * sizeof(double));
    double *R0 = (double *)calloc(nn, sizeof(double));
    double *U = (double *)calloc(nn, sizeof(double));
    double *G = (double *)calloc(nn, sizeof(double));
    double *B = (double *)malloc((size_t)m * (size_t)n * sizeof(double));
    double *c = (double *)calloc((size_t)n, sizeof(double));
    double *z = (double *)calloc((size_t)n, sizeof(double));
    int info = 0;
    if (sketch == 1) or_sketch_rows(m, n, A, lda, s, seed, Bs, s);
    else or_sketch_apply(m, n, A, lda, s, seed, Bs, s);
    info = (variant == 1) ? or_lu_r(s, n, Bs, s, R0, n, NULL) : or_householder_r(s, n, Bs, s, R0, n);
    if (!info) {
        or_trsm_ru(m, n, A, lda, R0, n, B, m);
        or_gram(m, n, B, m, G, n);
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t i = 0; i < m; ++i) acc += B[IDX(i, j, m)] * b[i];
            c[j] = acc;
        }
        int k = or_cholesky_upper(n, G, n, U, n);
        if (k) info = 2000 + k;
    }
    if (!info) {
        for (int64_t i = 0; i < n; ++i) {  /* U^T z = c */
            double acc = c[i];
            for (int64_t k = 0; k < i; ++k) acc -= U[IDX(k, i, n)] * z[k];
            z[i] = acc / U[IDX(i, i, n)];
        }
        for (int64_t i = n - 1; i >= 0; --i) {  /* U y = z (y into c) */
            double acc = z[i];
            for (int64_t k = i + 1; k < n; ++k) acc -= U[IDX(i, k, n)] * c[k];
            c[i] = acc / U[IDX(i, i, n)];
        }
        for (int64_t i = n - 1; i >= 0; --i) {  /* R0 x = y */
            double acc = c[i];
            for (int64_t k = i + 1; k < n; ++k) acc -= R0[IDX(i, k, n)] * x[k];
            x[i] = acc / R0[IDX(i, i, n)];
        }
    } else {
        for (int64_t i = 0; i < n; ++i) x[i] = NAN;
    }
    free(Bs); free(R0); free(U); free(G); free(B); free(c); free(z);
    return info;
}

/* CholeskyQR (npass = 1), CholeskyQR2 (npass = 2) and plain repeated passes, with an
 * optional diagonal shift on the first Gram matrix G (paper Algorithm sCholeskyQR3 uses a
 * shift with npass = 3): shift > 0 is added as given; shift < 0 adds the paper's suggested
 * 11 (m n + n (n + 1)) u ||A||_2^2 (Section 2.1) with ||A||_2^2 bounded above by ||G||_F
 * and u = 2^-52, the machine precision the paper defines in Section 4.1.
 * R = R_npass ... R_1.  Returns 0 or 1000*(pass+1) + k. */
int or_cholqr_n(int64_t m, int64_t n, const double *A, int64_t lda, int npass,
                double shift, double *Q, int64_t ldq, double *R, int64_t ldr) {
    size_t nn = (size_t)n * (size_t)n;
    double *W = (double *)malloc(nn * sizeof(double));
    double *Rk = (double *)malloc(nn * sizeof(double));
    double *Racc = (double *)calloc(nn, sizeof(double));
    double *T = (double *)malloc(nn * sizeof(double));
    int info = 0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < m; ++i) Q[IDX(i, j, ldq)] = A[IDX(i, j, lda)];
    for (int64_t k = 0; k < n; ++k) Racc[IDX(k, k, n)] = 1.0;
    for (int pass = 0; pass < npass && !info; ++pass) {
        or_gram(m, n, Q, ldq, W, n);
        if (pass == 0 && shift != 0.0) {
            double sh = shift;
            if (shift < 0.0)
                sh = 11.0 * ((double)m * (double)n + (double)n * (double)(n + 1)) * 0x1p-52 *
                     or_fro(n, W, n);
            for (int64_t k = 0; k < n; ++k) W[IDX(k, k, n)] += sh;
        }
        int c = or_cholesky_upper(n, W, n, Rk, n);
        if (c) { info = 1000 * (pass + 1) + c; break; }
        or_trsm_ru(m, n, Q, ldq, Rk, n, Q, ldq);
        or_trmm_upper(n, Rk, n, Racc, n, T, n);
        memcpy(Racc, T, nn * sizeof(double));
    }
    if (info) {
        fill_nan(m, n, Q, ldq);
        fill_nan(n, n, R, ldr);
    } else {
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) R[IDX(i, j, ldr)] = Racc[IDX(i, j, n)];
    }
    free(W); free(Rk); free(Racc); free(T);
    return info;
}

/* ------------------------------------------------------------------------------------
 * Accuracy metrics (paper Section 4.2): orthogonality ||Q^T Q - I||_F and residual
 * ||A - QR||_F / ||A||_F.  Every dot product and every sum of squares is accumulated in
 * double-double arithmetic (error-free TwoSum and fma-based TwoProd: Ogita, Rump, Oishi,
 * "Accurate sum and dot product", SISC 2005), so the metric's own rounding (about
 * 2u in relative terms) stays far below the quantities measured.
 * ------------------------------------------------------------------------------------ */
typedef struct { double hi, lo; } dd_t;

static inline void dd_add(dd_t *acc, double x) {
    double s = acc->hi + x;
    double bp = s - acc->hi;
    double err = (acc->hi - (s - bp)) + (x - bp);
    acc->hi = s;
    acc->lo += err;
}

static inline void dd_add_prod(dd_t *acc, double a, double b) {
    double p = a * b;
    double e = fma(a, b, -p);
    dd_add(acc, p);
    acc->lo += e;
}

static inline double dd_value(dd_t a) { return a.hi + a.lo; }

double or_orthogonality(int64_t m, int64_t n, const double *Q, int64_t ldq) {
    double *E = (double *)malloc((size_t)n * (size_t)n * sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < n; ++b)
        for (int64_t a = 0; a <= b; ++a) {
            dd_t acc = {0.0, 0.0};
            const double *qa = Q + IDX(0, a, ldq), *qb = Q + IDX(0, b, ldq);
            for (int64_t j = 0; j < m; ++j) dd_add_prod(&acc, qa[j], qb[j]);
            if (a == b) dd_add(&acc, -1.0);
            E[IDX(a, b, n)] = dd_value(acc);
        }
    dd_t f = {0.0, 0.0};
    for (int64_t b = 0; b < n; ++b)
        for (int64_t a = 0; a <= b; ++a) {
            double e = E[IDX(a, b, n)];
            dd_add_prod(&f, e, e);
            if (a != b) dd_add_prod(&f, e, e);
        }
    free(E);
    return sqrt(dd_value(f));
}

double or_residual(int64_t m, int64_t n, const double *A, int64_t lda, const double *Q,
                   int64_t ldq, const double *R, int64_t ldr) {
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    dd_t *num = (dd_t *)calloc((size_t)nthr, sizeof(dd_t));
    dd_t *den = (dd_t *)calloc((size_t)nthr, sizeof(dd_t));
#pragma omp parallel
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i)
            for (int64_t j = 0; j < n; ++j) {
                dd_t e = {0.0, 0.0};
                double a = A[IDX(i, j, lda)];
                dd_add(&e, a);
                for (int64_t k = 0; k < n; ++k) dd_add_prod(&e, -Q[IDX(i, k, ldq)], R[IDX(k, j, ldr)]);
                double ev = dd_value(e);
                dd_add_prod(&num[t], ev, ev);
                dd_add_prod(&den[t], a, a);
            }
    }
    dd_t nsum = {0.0, 0.0}, dsum = {0.0, 0.0};
    for (int t = 0; t < nthr; ++t) {
        dd_add(&nsum, num[t].hi); dd_add(&nsum, num[t].lo);
        dd_add(&dsum, den[t].hi); dd_add(&dsum, den[t].lo);
    }
    free(num); free(den);
    return sqrt(dd_value(nsum)) / sqrt(dd_value(dsum));
}

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------
 * Mixed precision (a reading of the benchmark's mixed configuration, not in the paper):
 * the sketch takes its normals rounded to FP32 or BF16 and A as FP32 (see
 * or_sketch_apply_lowp); the preconditioner apply A1 = A R0^{-1} and the first Gram
 * matrix take inputs rounded to FP32 (either input type of the sketch; the routines also
 * take BF16, which the method does not use); R0, R0^{-1}, the Cholesky factors, the R
 * products and the final CholeskyQR passes are FP64.  Roundings: FP64 -> FP32 round to
 * nearest even;
 * BF16 = round to nearest even of that FP32 value to 8 significant bits.  The low-precision
 * steps here are the exact (FP64-accumulated) sums of the rounded inputs; a device may
 * add FP32 accumulation error on top, bounded in the tests.
 * ------------------------------------------------------------------------------------ */
#define OR_FP32 1
#define OR_BF16 2

double or_round_fp32(double x) { return (double)(float)x; }

double or_round_bf16(double x) {
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan unchanged */
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb; /* round to nearest, ties to even, on the upper 16 bits */
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double or_round_p(int prec, double x) {
    return prec == OR_BF16 ? or_round_bf16(x) : or_round_fp32(x);
}

/* B = (1/sqrt(s)) * sum_j r(Z(i,j)) fp32(A(j,c)): the normal Z is first made an FP32
 * number (as the sketch defines it) and then rounded to the input type r; A enters as its
 * FP32 rounding for both input types.  (With BF16 inputs that FP32 value is carried as the
 * exact sum of three BF16 numbers, each product of a BF16 normal with one of them exact,
 * so the sketch loses no more of A than with FP32 inputs.) */
void or_sketch_apply_lowp(int prec, int64_t m, int64_t n, const double *A, int64_t lda,
                          int64_t s, uint64_t seed, double *B, int64_t ldb) {
    double rs = 1.0 / sqrt((double)s);
#pragma omp parallel
    {
        double *zrow = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
#pragma omp for schedule(dynamic, 1)
        for (int64_t i = 0; i < s; ++i) {
            for (int64_t j = 0; j < m; ++j)
                zrow[j] = or_round_p(prec, or_round_fp32(or_sketch_normal(seed, i, j)));
            for (int64_t c = 0; c < n; ++c) {
                double acc = 0.0;
                for (int64_t j = 0; j < m; ++j) acc += zrow[j] * or_round_fp32(A[IDX(j, c, lda)]);
                B[IDX(i, c, ldb)] = rs * acc;
            }
        }
        free(zrow);
    }
}

/* X = r(Y) r(Rinv) for upper-triangular Rinv, summed in FP64, then rounded to the input
 * type (the stored low-precision A1). */
void or_apply_rinv_lowp(int prec, int64_t m, int64_t n, const double *Y, int64_t ldy,
                        const double *Rinv, int64_t ldr, double *X, int64_t ldx) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int64_t c = 0; c < n; ++c) {
            double acc = 0.0;
            for (int64_t k = 0; k <= c; ++k)
                acc += or_round_p(prec, Y[IDX(i, k, ldy)]) * or_round_p(prec, Rinv[IDX(k, c, ldr)]);
            X[IDX(i, c, ldx)] = or_round_p(prec, acc);
        }
}

/* W = r(X)^T r(X), FP64 sums (both triangles). */
void or_gram_lowp(int prec, int64_t m, int64_t n, const double *X, int64_t ldx, double *W,
                  int64_t ldw) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < n; ++b)
        for (int64_t a = 0; a <= b; ++a) {
            double acc = 0.0;
            for (int64_t j = 0; j < m; ++j)
                acc += or_round_p(prec, X[IDX(j, a, ldx)]) * or_round_p(prec, X[IDX(j, b, ldx)]);
            W[IDX(a, b, ldw)] = acc;
            W[IDX(b, a, ldw)] = acc;
        }
}

/* Inverse of an upper-triangular T by substitution, column by column (T X = I). */
void or_trtri_upper(int64_t n, const double *T, int64_t ldt, double *X, int64_t ldx) {
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = n - 1; i >= 0; --i) {
            double acc = (i == j) ? 1.0 : 0.0;
            if (i > j) { X[IDX(i, j, ldx)] = 0.0; continue; }
            for (int64_t k = i + 1; k <= j; ++k) acc -= T[IDX(i, k, ldt)] * X[IDX(k, j, ldx)];
            X[IDX(i, j, ldx)] = acc / T[IDX(i, i, ldt)];
        }
}

/* The mixed-precision method with a fixed number of FP64 passes (1..3):
 *   B = lowp sketch;  R0 = R factor of B (FP64);  R0inv = R0^{-1} (FP64);
 *   A1 = fp32(A R0inv);  W1 = FP32 Gram of A1;  R1 = chol(W1)  (breakdown -> R01 = R0);
 *   R01 = R1 R0;  Q = A R01^{-1};  passes: W = Q^T Q, Rk = chol(W), Q = Q Rk^{-1},
 *   R = Rk ... R01.
 * The stage (A1, W1, R1) takes FP32 inputs for both input types of the sketch: a stage with
 * BF16 inputs could only help below cond(A) ~ 1e2.  Automatic mode (fp64_passes = 0) first
 * decides whether the stage is run at all: only if ||R0||_F ||R0^{-1}||_F u_p <= 1
 * (u_p = 2^-24, the stage's FP32), an upper bound of cond(R0) u_p, i.e. if the rounding of
 * A to FP32 perturbs A R0^{-1} by well under one.  Otherwise R01 = R0 and *lp_info = -1.
 * Returns info as or_rxr_cholqr (stages 3, 4 = first, further FP64 passes); *lp_info
 * receives the low-precision Cholesky's breakdown column (0 if none, -1 if the stage was
 * not run), *passes_out the number of FP64 passes completed. */
static double or_fro(int64_t n, const double *X, int64_t ldx) {
    double acc = 0.0;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i) acc += X[IDX(i, j, ldx)] * X[IDX(i, j, ldx)];
    return sqrt(acc);
}

int or_rxr_cholqr_mixed(int variant, int prec, int64_t m, int64_t n, const double *A,
                        int64_t lda, int64_t s, uint64_t seed, int fp64_passes, double *Q,
                        int64_t ldq, double *R, int64_t ldr, int *lp_info, int *passes_out) {
    size_t nn = (size_t)n * (size_t)n;
    double *B = (double *)malloc((size_t)s * (size_t)n * sizeof(double));
    double *R0 = (double *)calloc(nn, sizeof(double));
    double *R0inv = (double *)calloc(nn, sizeof(double));
    double *R1 = (double *)calloc(nn, sizeof(double));
    double *Racc = (double *)calloc(nn, sizeof(double));
    double *Rk = (double *)calloc(nn, sizeof(double));
    double *T = (double *)calloc(nn, sizeof(double));
    double *W = (double *)calloc(nn, sizeof(double));
    double *A1 = (double *)malloc((size_t)m * (size_t)n * sizeof(double));
    int info = 0, lp = 0, npass = 0;

    or_sketch_apply_lowp(prec, m, n, A, lda, s, seed, B, s);
    info = (variant == 1) ? or_lu_r(s, n, B, s, R0, n, NULL) : or_householder_r(s, n, B, s, R0, n);
    if (!info) {
        or_trtri_upper(n, R0, n, R0inv, n);
        int stage = 1;
        if (fp64_passes == 0) stage = or_fro(n, R0, n) * or_fro(n, R0inv, n) * 0x1p-24 <= 1.0;
        if (stage) {
            or_apply_rinv_lowp(OR_FP32, m, n, A, lda, R0inv, n, A1, m);
            or_gram_lowp(OR_FP32, m, n, A1, m, W, n);
            lp = or_cholesky_upper(n, W, n, R1, n);
        } else {
            lp = -1;
        }
        if (lp) memcpy(Racc, R0, nn * sizeof(double));
        else or_trmm_upper(n, R1, n, R0, n, Racc, n);
        or_trsm_ru(m, n, A, lda, Racc, n, Q, ldq);
        /* fp64_passes = 1..3: that many plain passes.  0 = automatic: per pass, with
         * W = Q^T Q, dev = ||W - I||_F; a Cholesky breakdown is retried with the shift
         * 11 (m n + n (n+1)) u ||W||_F on the diagonal (shifted CholeskyQR, paper
         * Section 2.1); another pass follows while dev > 1/2 or the shift was used, at
         * most three passes. */
        int maxp = fp64_passes > 0 ? fp64_passes : 3, more = 1, last_shifted = 0;
        for (int pass = 0; pass < maxp && more && !info; ++pass) {
            or_gram(m, n, Q, ldq, W, n);
            double dev2 = 0.0, w2 = 0.0;
            for (int64_t j = 0; j < n; ++j)
                for (int64_t i = 0; i < n; ++i) {
                    double d = W[IDX(i, j, n)] - (i == j ? 1.0 : 0.0);
                    dev2 += d * d;
                    w2 += W[IDX(i, j, n)] * W[IDX(i, j, n)];
                }
            int c = or_cholesky_upper(n, W, n, Rk, n), shifted = 0;
            if (c && fp64_passes == 0) {
                double shift = 11.0 * ((double)m * (double)n + (double)n * (double)(n + 1)) *
                               0x1p-52 * sqrt(w2);
                for (int64_t k = 0; k < n; ++k) W[IDX(k, k, n)] += shift;
                c = or_cholesky_upper(n, W, n, Rk, n);
                shifted = 1;
            }
            if (c) { info = (pass == 0 ? 3000 : 4000) + c; break; }
            or_trsm_ru(m, n, Q, ldq, Rk, n, Q, ldq);
            or_trmm_upper(n, Rk, n, Racc, n, T, n);
            memcpy(Racc, T, nn * sizeof(double));
            ++npass;
            last_shifted = shifted;
            if (fp64_passes == 0) more = shifted || !(sqrt(dev2) <= 0.5);
        }
        /* the pass budget ran out: the last allowed pass itself needed the shift, so its
         * output is not yet orthonormal */
        if (!info && fp64_passes == 0 && npass == maxp && last_shifted) info = 5000;
    }
    if (!info)
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i) R[IDX(i, j, ldr)] = Racc[IDX(i, j, n)];
    else {
        fill_nan(m, n, Q, ldq);
        fill_nan(n, n, R, ldr);
    }
    if (lp_info) *lp_info = lp;
    if (passes_out) *passes_out = npass;
    free(B); free(R0); free(R0inv); free(R1); free(Racc); free(Rk); free(T); free(W); free(A1);
    return info;
}
