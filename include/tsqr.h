/*
 * tsqr.h -- C ABI of libtsqr: randomized XR-preconditioned CholeskyQR of a tall and
 * skinny FP64 matrix (Fan, Guo, Lin, "A Novel Randomized XR-Based Preconditioned
 * CholeskyQR Algorithm", arXiv 2111.11148) on one AMD Instinct MI355X (gfx950).
 *
 * Problem (paper Section 1, QR equation; Section 2 opening): given a full-rank
 * A (m x n, m >= n), return the thin factorization A = Q R with Q^T Q = I (m x n) and R
 * upper triangular (n x n) with a positive diagonal.
 *
 * Conventions for every entry point
 *   - matrices are column-major with a leading dimension: element (i, j) of X is
 *     X[i + j*ldx] (LAPACK convention); leading dimensions are counted in elements;
 *   - every matrix, workspace and info pointer is a DEVICE pointer owned by the caller;
 *     the library keeps no pointer after the call returns;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream); all work is
 *     enqueued on it in order and the host does not wait for it;
 *   - return value: 0 on success; -i if the i-th argument (1-based) is invalid, detected
 *     before any work is enqueued; TSQR_ERR_HIP if a HIP call fails; TSQR_ERR_WORKSPACE if
 *     the workspace is too small; TSQR_ERR_UNSUPPORTED for sizes the library does not
 *     implement;
 *   - numerical breakdown is reported asynchronously through `d_info` (device int):
 *     0 = success; 1000*stage + k = zero, non-positive or NaN pivot at column k (1-based)
 *     of stage 1 (the sketch factor R0), 2 (first Cholesky R1) or 3 (second Cholesky R2).
 *     After a breakdown every entry of Q and R is NaN.  Only the first breakdown is kept.
 *
 * The Gaussian sketch S (s x m) of paper Section 2.3 is S = Z / sqrt(s) with Z(i, j) ~
 * N(0,1) regenerated on the fly and never stored.  Stream: key = (low, high) 32-bit
 * halves of `seed`; one Philox4x32-10 call (Salmon et al., SC'11) with counter
 * (low32(p), high32(p), i, 0) yields Z(i, 4p .. 4p+3): words (w0, w1) give columns 4p and
 * 4p+1, (w2, w3) give 4p+2 and 4p+3 by the Box-Muller transform of the 24-bit uniforms
 * u = ((wa >> 8) + 1) 2^-24 and t = (wb >> 8) 2^-24: rad = sqrt(-2 ln u),
 * (rad cos 2 pi t, rad sin 2 pi t).  The device evaluates the transform in single precision
 * (entries of Z are FP32 numbers, exact in FP64); the integer stream is bit-exact.
 */
#ifndef TSQR_H
#define TSQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSQR_OK 0
#define TSQR_ERR_HIP (-100)
#define TSQR_ERR_WORKSPACE (-101)
#define TSQR_ERR_UNSUPPORTED (-102)

#define TSQR_VARIANT_RQR 0 /* R0 from Householder QR of the sketch */
#define TSQR_VARIANT_RLU 1 /* R0 from partial-pivot LU of the sketch */

/* ------------------------------------------------------------------------------------
 * Whole factorization
 * ------------------------------------------------------------------------------------ */

/* rQR-CholeskyQR (paper Algorithm rQR-CholeskyQR with the Gaussian sketch of Section 2.3)
 * followed by one more CholeskyQR pass (paper Algorithm CholeskyQR2, second line):
 *   B = S A (s x n);  R0 = R factor of B (Householder, diag > 0);  A1 = A R0^{-1};
 *   R1 = chol(A1^T A1);  Q1 = A1 R1^{-1};  R2 = chol(Q1^T Q1);  Q = Q1 R2^{-1};
 *   R = R2 (R1 R0).
 * m, n        : rows and columns of A, 1 <= n <= m, n <= 1024 (TSQR_ERR_UNSUPPORTED
 *               above).                                                    (args 1, 2)
 * A, lda      : input, read only, lda >= m.                               (args 3, 4)
 * sketch_rows : s, rows of the sketch, n <= s <= 8192 (the paper uses 2n). (arg 5)
 * seed        : sketch seed (see the stream definition above).            (arg 6)
 * Q           : output m x n with leading dimension m; must not overlap A. (arg 7)
 * R           : output n x n upper (strict lower part zeroed), leading dimension n;
 *               NULL skips forming R (the R-less variant of the paper's footnote to
 *               Algorithm CholeskyQR2).                                    (arg 8)
 * stream      : HIP stream.                                                (arg 9)
 * Scratch memory is taken from HIP's stream-ordered allocator on `stream`; breakdown
 * is visible only as NaN in Q and R (use tsqr_rxr_cholqr_ws for an info word). */
int tsqr_rqr_cholqr(int64_t m, int64_t n, const double* A, int64_t lda, int64_t sketch_rows,
                    uint64_t seed, double* Q, double* R, void* stream);

/* rLU-CholeskyQR (paper Algorithm rLU-CholeskyQR): as tsqr_rqr_cholqr with R0 taken from
 * Gaussian elimination with partial pivoting of B (pivot = first largest |b_ik|),
 * R0 = diag(sign u_kk) U.  Same arguments and codes. */
int tsqr_rlu_cholqr(int64_t m, int64_t n, const double* A, int64_t lda, int64_t sketch_rows,
                    uint64_t seed, double* Q, double* R, void* stream);

/* Bytes of device workspace needed by tsqr_rxr_cholqr_ws for these sizes (0 if the sizes
 * are invalid). */
size_t tsqr_workspace_bytes(int64_t m, int64_t n, int64_t sketch_rows);

/* Explicit-workspace form (no allocation inside; suitable for stream capture of the
 * kernels, reuse across calls and info reporting):
 *   variant (1): TSQR_VARIANT_RQR or TSQR_VARIANT_RLU;
 *   m, n, A, lda, sketch_rows, seed (2-7): as above;
 *   extra_pass (8): nonzero runs the extra CholeskyQR pass (R = R2 R1 R0), zero stops
 *     after the first pass (Q = Q1, R = R1 R0, the paper's algorithm as printed);
 *   Q, ldq (9, 10): output, ldq >= m, must not overlap A;
 *   R, ldr (11, 12): output or NULL, ldr >= n;
 *   work, work_bytes (13, 14): device workspace of at least tsqr_workspace_bytes() bytes,
 *     256-byte aligned; its contents on entry are ignored;
 *   d_info (15): device int written with the breakdown code, or NULL;
 *   stream (16). */
int tsqr_rxr_cholqr_ws(int variant, int64_t m, int64_t n, const double* A, int64_t lda,
                       int64_t sketch_rows, uint64_t seed, int extra_pass, double* Q,
                       int64_t ldq, double* R, int64_t ldr, void* work, size_t work_bytes,
                       int* d_info, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): tsqr_rxr_cholqr_ws with its workspace
 * taken from a fixed device array of TSQR_STATIC_SCRATCH_BYTES bytes that the library
 * holds on each GPU it runs on until the process ends.  Nothing is allocated and no
 * library routine that allocates is called.  Same arguments and codes as
 * tsqr_rxr_cholqr_ws without (work, work_bytes); d_info may be NULL (the info word then
 * lives in the array).  Sizes whose workspace (tsqr_workspace_bytes) exceeds
 * TSQR_STATIC_SCRATCH_BYTES return TSQR_ERR_WORKSPACE before any work is enqueued: every
 * n <= 128 with s <= 256 fits, at any m.  Every call on one GPU shares that GPU's array:
 * calls that overlap in time on one GPU (on different streams, or from several host
 * threads) race and give wrong results; calls on one stream are ordered and safe.  Each
 * call overwrites everything it reads from the array before reading it. */
#define TSQR_STATIC_SCRATCH_BYTES (72ull << 20)
int tsqr_rxr_cholqr_noalloc(int variant, int64_t m, int64_t n, const double* A, int64_t lda,
                            int64_t sketch_rows, uint64_t seed, int extra_pass, double* Q,
                            int64_t ldq, double* R, int64_t ldr, int* d_info, void* stream);

/* Row-extraction sketch (paper Section 2.3, "Row Extraction", the sketch of the paper's
 * experiments): rQR/rLU-CholeskyQR with B = P A, P selecting s rows drawn independently,
 * each uniformly from the m rows (the sampling of Theorem "Equal Probability Case"; a row
 * may repeat).  Draw i: Philox4x32-10 with key (seed lo, seed hi) and counter (i lo, i hi,
 * 0, 1); with w = word0 + 2^32 word1, row r_i = floor(w m / 2^64).  Arguments, codes,
 * workspace (tsqr_workspace_bytes) and info as tsqr_rxr_cholqr_ws.  An A whose mass
 * sits in few rows (the paper's [I; 0] example) can give a rank-deficient sample: a
 * breakdown of the small factorization, info = 1000 + k. */
int tsqr_rxr_cholqr_rows_ws(int variant, int64_t m, int64_t n, const double* A, int64_t lda,
                            int64_t sketch_rows, uint64_t seed, int extra_pass, double* Q,
                            int64_t ldq, double* R, int64_t ldr, void* work, size_t work_bytes,
                            int* d_info, void* stream);

/* ------------------------------------------------------------------------------------
 * Least squares min ||A x - b||_2 preconditioned by the sketch's R factor (paper Section
 * 5.2, Algorithm "LS solver preconditioned by randomized R factor"; its R_1 is R0 here):
 *   R0 = R factor of the sketch (QR or LU of the Gaussian or row-extraction sketch);
 *   B = A R0^{-1} (right-side TRSM);  G = B^T B = U^T U (Cholesky);  c = B^T b;
 *   y = U^{-1} U^{-T} c (the normal equation of B y = b);  x = R0^{-1} y.
 * ------------------------------------------------------------------------------------ */
#define TSQR_SKETCH_GAUSSIAN 0
#define TSQR_SKETCH_ROWS 1

/* Bytes of workspace for tsqr_lstsq_ws (0 if the sizes are invalid); it holds B (m x n). */
size_t tsqr_lstsq_workspace_bytes(int64_t m, int64_t n, int64_t sketch_rows);

/*   variant (1): TSQR_VARIANT_RQR or TSQR_VARIANT_RLU;  sketch (2): TSQR_SKETCH_*;
 *   m, n, A, lda (3-6): as tsqr_rxr_cholqr_ws;  b (7): device vector of m doubles;
 *   sketch_rows, seed (8, 9);  x (10): device output, n doubles;
 *   work, work_bytes (11, 12): at least tsqr_lstsq_workspace_bytes() bytes;
 *   d_info (13): device int: 1000 + k (small factorization), 2000 + k (Cholesky of G),
 *     x then NaN; or NULL;  stream (14).
 * Codes: -i for argument i (m < n is -3), TSQR_ERR_WORKSPACE, TSQR_ERR_UNSUPPORTED
 * (n > 1024), TSQR_ERR_HIP. */
int tsqr_lstsq_ws(int variant, int sketch, int64_t m, int64_t n, const double* A, int64_t lda,
                  const double* b, int64_t sketch_rows, uint64_t seed, double* x, void* work,
                  size_t work_bytes, int* d_info, void* stream);

/* ------------------------------------------------------------------------------------
 * CholeskyQR family (paper Section 2.1: Algorithms CholeskyQR, CholeskyQR2 and
 * sCholeskyQR3), the baselines the paper compares against, on the same kernels.
 * ------------------------------------------------------------------------------------ */
#define TSQR_ALGO_CHOLQR 1   /* one pass: W = A^T A, R = chol(W), Q = A R^{-1} */
#define TSQR_ALGO_CHOLQR2 2  /* two passes, R = R2 R1 */
#define TSQR_ALGO_SCHOLQR3 3 /* first Cholesky of W + shift I, then two passes, R = R3 R2 R1 */

/* Bytes of workspace for tsqr_cholqr_ws (0 if the sizes are invalid). */
size_t tsqr_cholqr_workspace_bytes(int64_t m, int64_t n);

/*   algo (1): TSQR_ALGO_*;
 *   m, n, A, lda (2-5): as tsqr_rxr_cholqr_ws;
 *   shift (6): sCholeskyQR3 only: >= 0 is added to the first Gram matrix's diagonal as
 *     given (the paper's experiments use 1e-15 for ||A||_2 = 1); < 0 adds the suggested
 *     11 (m n + n (n + 1)) u ||A||_2^2 with u = 2^-52 (the machine precision of Section
 *     4.1) and ||A||_2^2 bounded above by ||A^T A||_F (computed on the device, no host
 *     wait); NaN is an argument error;
 *   Q, ldq (7, 8), R, ldr (9, 10): outputs as tsqr_rxr_cholqr_ws;
 *   work, work_bytes (11, 12): at least tsqr_cholqr_workspace_bytes(m, n) bytes;
 *   d_info (13): device int, 1000 * pass + k when pass `pass`'s Cholesky breaks down at
 *     column k (Q and R then NaN), or NULL;  stream (14). */
int tsqr_cholqr_ws(int algo, int64_t m, int64_t n, const double* A, int64_t lda, double shift,
                   double* Q, int64_t ldq, double* R, int64_t ldr, void* work, size_t work_bytes,
                   int* d_info, void* stream);

/* ------------------------------------------------------------------------------------
 * Mixed precision
 * ------------------------------------------------------------------------------------ */
#define TSQR_LOWP_FP32 1 /* inputs rounded to FP32, FP32 matrix cores, FP32 accumulation */
#define TSQR_LOWP_BF16 2 /* inputs rounded to BF16 (RNE of the FP32 value), FP32 accumulation;
                            the sketch's A excepted (see tsqr_sketch_lowp) and, in
                            tsqr_rxr_cholqr_mixed_ws, the stage after the sketch */

/* Randomized XR-preconditioned CholeskyQR with the data-heavy preconditioning steps in low
 * precision and the orthogonalising passes in FP64 (the paper's framework, Section 2.2,
 * with an inexact preconditioner as analysed in Appendix A):
 *   B = S A on the `lowp` matrix cores (as tsqr_sketch_lowp: FP32 accumulation over at
 *     most 64 rows, FP64 partial sums);
 *   R0 = R factor of B in FP64 (Householder or LU as `variant`);
 *   R0^{-1} explicitly in FP64 (triangular solve of the identity), rounded to FP32;
 *   A1 = A R0^{-1} and W1 = A1^T A1 with FP32 inputs for either `lowp` (W1 summed in FP64;
 *     with BF16 inputs this stage could only save an FP64 pass below cond(A) ~ 1e2);
 *   R1 = chol(W1) in FP64; R01 = R1 R0 (or R0 alone if this Cholesky breaks down: the
 *     low-precision factor is then discarded and the FP64 passes start from R0);
 *   FP64 CholeskyQR passes on A R01^{-1}: Q1 = A R01^{-1} by FP64 substitution from the
 *     FP64 A, W = Q1^T Q1, Rk = chol(W), Q = Q1 Rk^{-1}, R = Rk ... R01.
 * fp64_passes (arg 9): 1, 2 or 3 fixed FP64 passes, or 0 = automatic: a further pass runs
 *   while the Gram matrix of a pass's input deviates from I by more than 1/2 in Frobenius
 *   norm or its Cholesky factorization broke down (it is then retried with the shift
 *   11 (m n + n (n + 1)) u ||W||_F on the diagonal, u = 2^-52, the shifted CholeskyQR of
 *   Section 2.1), at most 3 passes.  The automatic mode also skips the low-precision
 *   A1/W1/R1 stage (R01 = R0, low precision for the sketch only) unless
 *   ||R0||_F ||R0^{-1}||_F u_p <= 1 (u_p = 2^-24, the stage's FP32): beyond that bound on
 *   cond(R0) u_p the stage cannot save an FP64 pass.  Every decision is taken on
 *   the device (the stage's and the passes' kernels are enqueued and return at once when
 *   not needed), so no mode waits on the host and every mode may be captured into a graph.
 *   If the third pass of the automatic mode still needed the shifted retry, the pass
 *   budget ran out: *d_info = 5000 and Q and R are NaN.
 * d_report (arg 16): NULL, or two device ints receiving [0] the number of FP64 passes
 *   run and [1] 1 if the low-precision stage ran (0 if the automatic mode skipped it).
 * lowp (arg 2): TSQR_LOWP_FP32 or TSQR_LOWP_BF16.  Other arguments as in
 * tsqr_rxr_cholqr_ws (shifted by one position); info stages 3 and 4 are the FP64 passes.
 * Workspace: tsqr_mixed_workspace_bytes(m, n, s, lowp) bytes (the same for either lowp).
 * n <= 256 (the low-precision kernels; TSQR_ERR_UNSUPPORTED above). */
size_t tsqr_mixed_workspace_bytes(int64_t m, int64_t n, int64_t sketch_rows, int lowp);
int tsqr_rxr_cholqr_mixed_ws(int variant, int lowp, int64_t m, int64_t n, const double* A,
                             int64_t lda, int64_t sketch_rows, uint64_t seed, int fp64_passes,
                             double* Q, int64_t ldq, double* R, int64_t ldr, void* work,
                             size_t work_bytes, int* d_info, int* d_report, void* stream);

/* Low-precision steps of the mixed variant (step-wise validation):
 *   tsqr_sketch_lowp: B = S A (s x n FP64, ldb >= s) with the entries of S rounded to
 *     `lowp` and those of A rounded to FP32 (both types), FP32 accumulation over at most
 *     64 rows, FP64 partial sums; workspace tsqr_sketch_workspace_bytes(m, n, s).  With
 *     BF16 the FP32 value of each entry of A is split exactly into three BF16 terms, each
 *     multiplied by the BF16 normal on the BF16 matrix cores (products exact in FP32):
 *     the sketch then costs three BF16 products per term, far below the normals'
 *     generation, and keeps A to FP32 accuracy, so it preconditions as well as the FP32
 *     sketch (a single BF16 rounding of A would leave cond(A R0^{-1}) near cond(A) 2^-8).
 *   tsqr_apply_rinv_lowp: X = r(Y) r(Rinv) for upper-triangular Rinv (n x n FP64, rounded
 *     inside), FP32 accumulation; X (m x n, ldx >= m) holds FP32 or BF16 elements (2-byte
 *     BF16 bit patterns); workspace tsqr_rinv_lowp_bytes(n, lowp).
 *   tsqr_gram_lowp: W = X^T X (both triangles, FP64) for X in `lowp` elements as written
 *     by tsqr_apply_rinv_lowp; FP32 accumulation over 64 rows, FP64 partial sums;
 *     workspace tsqr_gram_workspace_bytes(m, n). */
int tsqr_sketch_lowp(int lowp, int64_t m, int64_t n, const double* A, int64_t lda, int64_t s,
                     uint64_t seed, double* B, int64_t ldb, void* work, size_t work_bytes,
                     void* stream);
size_t tsqr_rinv_lowp_bytes(int64_t n, int lowp);
int tsqr_apply_rinv_lowp(int lowp, int64_t m, int64_t n, const double* Y, int64_t ldy,
                         const double* Rinv, int64_t ldr, void* X, int64_t ldx, void* work,
                         size_t work_bytes, void* stream);
int tsqr_gram_lowp(int lowp, int64_t m, int64_t n, const void* X, int64_t ldx, double* W,
                   int64_t ldw, void* work, size_t work_bytes, void* stream);

/* ------------------------------------------------------------------------------------
 * Batched factorizations: many independent problems of uneven sizes in one pass
 * ------------------------------------------------------------------------------------
 * Each problem is factored exactly as by tsqr_rxr_cholqr_ws with extra_pass = 1 (the
 * method of the paper's Algorithm rQR- or rLU-CholeskyQR with the Gaussian sketch of
 * Section 2.3 and one more CholeskyQR pass); the split-K blockings differ from the
 * single-problem calls, so results agree with them to rounding, not bitwise.
 * Limits: 1 <= n <= 128, n <= s <= 512 (s <= 256 when n > 64), m >= n; any other problem
 * makes the create call return -4.
 * Precision: TSQR_BATCH_FP64 runs every step in FP64; TSQR_LOWP_FP32 or TSQR_LOWP_BF16
 * computes the sketch S A on that type's matrix cores (normals in that type, A as its
 * FP32 rounding) with FP32 accumulation flushed into FP64 every 64 rows (as
 * tsqr_sketch_lowp) and every later step in FP64, the mixed variant with the low
 * precision in the sketch alone. */
#define TSQR_BATCH_FP64 0
typedef struct {
  int64_t m, n;        /* rows and columns of A */
  int64_t lda;         /* leading dimension of A (>= m) */
  int64_t s;           /* sketch rows */
  uint64_t seed;       /* sketch seed (stream as for the single-problem calls) */
  const double* A;     /* device, read only */
  double* Q;           /* device output, ld ldq >= m, must not overlap A */
  int64_t ldq;
  double* R;           /* device output (ld ldr >= n) or NULL */
  int64_t ldr;
} tsqr_problem;

typedef struct tsqr_batch tsqr_batch; /* opaque plan */

/* Blocking of a batch plan: rows of A per split-K workgroup of the sketch and of the Gram
 * kernels (multiples of 64, >= 1024), 16-row tiles per triangular-solve workgroup (>= 32). */
typedef struct {
  int64_t sketch_rows;
  int64_t gram_rows;
  int trsm_tiles;
} tsqr_batch_tuning;

/* Workspace bytes for a batch (0 if any problem is invalid); enough for every tuning.
 * `problems` is a host array. */
size_t tsqr_batched_workspace_bytes(int64_t count, const tsqr_problem* problems);

/* Plan a batch: groups the problems by width, sizes their blockings, lays out `work` and
 * uploads the problem descriptors and work lists into it (synchronously).  Arguments:
 * variant (1), precision (2: TSQR_BATCH_FP64, TSQR_LOWP_FP32 or TSQR_LOWP_BF16), count (3),
 * problems (4, host array, not kept), work / work_bytes (5, 6), d_info (7: device
 * int[count], one breakdown code per problem as for tsqr_rxr_cholqr_ws), tuning (8: NULL
 * for the defaults 2048 / 2048 / 64), out (9: receives the plan).  The plan refers to
 * `work`, `d_info` and the problems' device buffers: they must stay valid and unmoved
 * while the plan is used. */
int tsqr_batched_create(int variant, int precision, int64_t count, const tsqr_problem* problems,
                        void* work, size_t work_bytes, int* d_info,
                        const tsqr_batch_tuning* tuning, tsqr_batch** out);

/* Autotuner: plans and runs the batch with candidate blockings (coordinate search over
 * the sketch rows, the Gram rows and the solve tiles, each from four values) and returns
 * the fastest in *best and its time per run in *best_ms (may be NULL).  Runs the batch
 * (writes Q, R and d_info) and waits for the stream: call it outside any capture.
 * Arguments as tsqr_batched_create up to d_info, then stream (8), best (9), best_ms (10). */
int tsqr_batched_autotune(int variant, int precision, int64_t count,
                          const tsqr_problem* problems, void* work, size_t work_bytes, int* d_info,
                          void* stream, tsqr_batch_tuning* best, double* best_ms);

/* The same search timing the persistent launch (tsqr_batched_run_persistent), over coarser
 * candidates (2048 to 16384 rows, 64 to 512 tiles): its tasks pay a publish and, for the
 * solves, an operand staging each. */
int tsqr_batched_autotune_persistent(int variant, int precision, int64_t count,
                                     const tsqr_problem* problems, void* work, size_t work_bytes,
                                     int* d_info, void* stream, tsqr_batch_tuning* best,
                                     double* best_ms);

/* Enqueue the whole batch on `stream`.  Kernel launches only (no allocation, copy or host
 * synchronisation), so a stream capture of this call records the batch as one graph. */
int tsqr_batched_run(tsqr_batch* plan, void* stream);

/* The same batch as ONE persistent kernel (preceded by one small kernel that clears its
 * counters): one workgroup per compute unit takes tasks from a queue in the plan's order
 * (every sketch task, then the solves by R0, the first Gram matrices, the solves by R1,
 * the second Gram matrices, the solves by R2); per-problem dependency counters in the
 * workspace let a task start as soon as its own problem's previous step is complete, and
 * the workgroup that completes a problem's last split-K task finishes that step (the
 * fixed-order reduction, the small factorization, the R product).  Results agree with
 * tsqr_batched_run to rounding (different reduction order) and are reproducible run to
 * run.  Kernel launches only, so it may be captured into a graph.  If the scheduler's
 * bounded wait ever gave up, every problem's info is 9000. */
int tsqr_batched_run_persistent(tsqr_batch* plan, void* stream);

/* The same, with the scheduler's time accounted (measurement): d_stats is NULL or 18
 * device counters (unsigned 64-bit, caller-zeroed, accumulated) of wall-clock ticks at
 * 100 MHz summed over the workgroups, per task kind k (0 sketch, 1-3 the solves by R0,
 * R1, R2, 4-5 the Gram matrices 1, 2): [3k] waiting for the problem's previous step,
 * [3k+1] the task itself, [3k+2] the finishing step (and publishing) after it. */
int tsqr_batched_run_persistent_timed(tsqr_batch* plan, unsigned long long* d_stats,
                                      void* stream);

/* Number of kernel launches one run of tsqr_batched_run enqueues (one per phase and width
 * class), and number of tasks of the persistent schedule. */
int tsqr_batched_launches(const tsqr_batch* plan);
int tsqr_batched_tasks(const tsqr_batch* plan);

void tsqr_batched_destroy(tsqr_batch* plan);

/* ------------------------------------------------------------------------------------
 * Steps of the method, one entry point per step (used for step-wise validation)
 * ------------------------------------------------------------------------------------ */

/* Row-extraction sketch (paper Section 2.3): B(i, :) = A(r_i, :) with the draws of
 * tsqr_rxr_cholqr_rows_ws; B is s x n (ldb >= s), an exact copy (no arithmetic).
 * Codes: -1 m < 1, -2 n < 1, -3 A NULL, -4 lda < m, -5 s outside [1, 8192], -7 B NULL,
 * -8 ldb < s. */
int tsqr_sketch_rows(int64_t m, int64_t n, const double* A, int64_t lda, int64_t s,
                     uint64_t seed, double* B, int64_t ldb, void* stream);

/* Sketch (paper Section 2.3, Gaussian ensemble): B = S A, B is s x n (ldb >= s).  The
 * sum over the m rows is split into row blocks whose partial sums are added in a fixed
 * order (deterministic).  Workspace: tsqr_sketch_workspace_bytes(m, n, s). */
size_t tsqr_sketch_workspace_bytes(int64_t m, int64_t n, int64_t s);
int tsqr_sketch(int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed,
                double* B, int64_t ldb, void* work, size_t work_bytes, void* stream);

/* R factor of the s x n sketch (paper Algorithms rQR/rLU-CholeskyQR, the sketch's
 * factorization):
 * variant TSQR_VARIANT_RQR = Householder QR (LAPACK reflector convention), RLU = partial
 * pivot LU; the result is sign-normalised, R0 = diag(sign d_k) * (R or U), and written as
 * an n x n upper matrix (strict lower part zeroed, ldr >= n).  A zero or NaN diagonal at
 * column k sets *d_info = 1000 + k (if *d_info was 0) and R0(k,k) = NaN.
 * Workspace (args 9, 10): tsqr_sketch_factor_workspace_bytes(s, n) bytes (a working copy
 * of B and the blocked factorization's reflector block). */
size_t tsqr_sketch_factor_workspace_bytes(int64_t s, int64_t n);
int tsqr_sketch_factor(int variant, int64_t s, int64_t n, const double* B, int64_t ldb,
                       double* R0, int64_t ldr, int* d_info, void* work, size_t work_bytes,
                       void* stream);

/* Right-side upper triangular solve X = Y T^{-1} by row-wise substitution (the Q = A R^{-1}
 * of paper Algorithm CholeskyQR; row-wise backward stable, no explicit inverse).
 * Y, X: m x n (ldy, ldx >= m); X may be the same buffer as Y with ldx == ldy (in place);
 * T: n x n upper, only its upper triangle is read.  n <= 1024 (above 128 columns the
 * solve runs by 128-column blocks with an MFMA update between them).
 * Workspace (args 9, 10): tsqr_trsm_workspace_bytes(n) bytes (a transposed copy of T). */
size_t tsqr_trsm_workspace_bytes(int64_t n);
int tsqr_trsm(int64_t m, int64_t n, const double* Y, int64_t ldy, const double* T, int64_t ldt,
              double* X, int64_t ldx, void* work, size_t work_bytes, void* stream);

/* Gram matrix W = X^T X (paper Algorithm CholeskyQR), both triangles written
 * (ldw >= n).  Split over row blocks, fixed-order reduction.  n <= 1024.
 * Workspace: tsqr_gram_workspace_bytes(m, n). */
size_t tsqr_gram_workspace_bytes(int64_t m, int64_t n);
int tsqr_gram(int64_t m, int64_t n, const double* X, int64_t ldx, double* W, int64_t ldw,
              void* work, size_t work_bytes, void* stream);

/* Cholesky W = R^T R (paper Algorithm CholeskyQR): reads the upper triangle of
 * W, writes upper R (strict lower part zeroed).  A pivot that is not positive (or NaN)
 * at column k sets *d_info = 1000*stage + k (if *d_info was 0) and makes R NaN from
 * column k on.  R may be W itself (ldr == ldw, in place); no other overlap.  n <= 8192.
 * work, work_bytes: unused (the factorization runs in R); NULL and 0 are accepted. */
int tsqr_potrf(int64_t n, const double* W, int64_t ldw, double* R, int64_t ldr, int stage,
               int* d_info, void* work, size_t work_bytes, void* stream);

/* C = A B for upper triangular n x n A and B (the R-factor products of paper Algorithms
 * rQR-CholeskyQR and CholeskyQR2).  C must not overlap A or B. */
int tsqr_trmm_upper(int64_t n, const double* A, int64_t lda, const double* B, int64_t ldb,
                    double* C, int64_t ldc, void* stream);

/* ------------------------------------------------------------------------------------
 * Generator access (validation of the sketch stream)
 * ------------------------------------------------------------------------------------ */

/* d_out[4e .. 4e+3] = Philox4x32-10(counter d_ctr[4e .. 4e+3], key (low32(seed),
 * high32(seed))) for e < count.  Device pointers. */
int tsqr_philox4x32_10(int64_t count, const uint32_t* d_ctr, uint64_t seed, uint32_t* d_out,
                       void* stream);

/* Z(i0 + a, j0 + b) -> Zout[a + b*ldz] for a < ni, b < nj: the N(0,1) entries of the
 * sketch before the 1/sqrt(s) scaling, exactly as the sketch kernel generates them. */
int tsqr_sketch_normals(uint64_t seed, int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                        double* Zout, int64_t ldz, void* stream);

/* ------------------------------------------------------------------------------------
 * Accuracy metrics and roofline probes (measurement; not part of the factorization)
 * ------------------------------------------------------------------------------------ */

/* The paper's two accuracy measures (Section 4.2), evaluated with double-double
 * accumulation (error-free FMA products, two-sum additions) in a fixed summation order:
 *   d_out[0] = ||Q^T Q - I||_F,   d_out[1] = ||A - Q R||_F / ||A||_F.
 * A plain FP64 sum over m rows would carry an error near sqrt(m) u, above the values
 * being measured once m is large; here each Gram entry and each entry of A - Q R is
 * accurate to about m u^2 of its terms, so both results have essentially full precision.
 * m, n        : rows and columns of Q (and A), m >= 1, 1 <= n <= 65536.   (args 1, 2)
 * A, lda      : the factorized matrix, lda >= m; NULL skips the residual (d_out[1] =
 *               NaN).                                                      (args 3, 4)
 * Q, ldq      : m x n, ldq >= m.                                           (args 5, 6)
 * R, ldr      : n x n as returned (every entry is used), ldr >= n; NULL skips the
 *               residual.                                                   (args 7, 8)
 * d_out       : two device doubles.                                        (arg 9)
 * work        : device workspace of tsqr_metrics_workspace_bytes(m, n) bytes (0 for
 *               invalid sizes); TSQR_ERR_WORKSPACE if smaller or NULL.     (args 10, 11) */
size_t tsqr_metrics_workspace_bytes(int64_t m, int64_t n);
int tsqr_metrics(int64_t m, int64_t n, const double* A, int64_t lda, const double* Q,
                 int64_t ldq, const double* R, int64_t ldr, double* d_out, void* work,
                 size_t work_bytes, void* stream);

/* Attainable-bandwidth probe: one pass of a plain streaming kernel with 16-byte accesses
 * over `bytes` bytes (rounded down to a multiple of 16): kind 0 reads src, 1 writes dst,
 * 2 copies src to dst.  Launch shape: wgs_per_cu workgroups of 256 threads per compute
 * unit (1..64), `unroll` words (1, 2, 4, 8) in flight per thread per loop trip, and
 * nontemporal != 0 for streaming stores.  Device pointers, 16-byte aligned; d_sink is one
 * device double that the read probe may write (it keeps the loads from being removed).
 * Errors: -1 kind, -2 src NULL (kinds 0, 2), -3 dst NULL (kinds 1, 2), -4 bytes < 16,
 * -5 wgs_per_cu, -6 unroll, -8 d_sink. */
int tsqr_probe_stream(int kind, const void* src, void* dst, size_t bytes, int wgs_per_cu,
                      int unroll, int nontemporal, double* d_sink, void* stream);

/* Attainable matrix-core rate probe: `chains` (4, 8, 16) independent accumulator chains
 * per wavefront, `iters` MFMAs each, on waves_per_simd (1, 2, 4, 8) workgroups of four
 * wavefronts per compute unit.  kind 0: FP64 16x16x4, 1: FP32 16x16x4, 2: BF16 16x16x32,
 * 3: BF16 32x32x16 (FP32 accumulation for the BF16 forms), 4: FP64 16x16x4 with random
 * operands drawn afresh at every step (kinds 0-3 keep their operands fixed).  *flops (host) is set to the
 * flops of the launch (2 per multiply-add).  Errors: -1 kind, -2 waves_per_simd, -3 chains,
 * -4 iters < 1, -5 d_sink NULL, -6 flops NULL. */
int tsqr_probe_mfma(int kind, int waves_per_simd, int chains, int64_t iters, double* d_sink,
                    double* flops, void* stream);

/* ------------------------------------------------------------------------------------
 * Phase timing (tracing)
 * ------------------------------------------------------------------------------------ */

/* While enabled, the whole-factorization entry points record a pair of HIP events on
 * their stream around every kernel they launch (named "sketch", "sketch_reduce",
 * "sketch_qr" or "sketch_lu", "trsm_prep_r0", "trsm_r0", "gram1", "gram1_reduce", "potrf1",
 * "trsm_prep_r1", "trsm_r1", "gram2", "gram2_reduce", "potrf2", "trsm_prep_r2", "trsm_r2",
 * "trmm", "poison"; the "trsm_prep" phases prepare the triangular factor's operand tiles,
 * the "trsm" phases are the solves themselves).  tsqr_profile_start()
 * clears the records and enables recording; tsqr_profile_stop() disables it, waits for
 * the recorded events and returns the number of records (or TSQR_ERR_HIP);
 * tsqr_profile_record(i) returns the i-th record's name (static storage) and duration in
 * milliseconds (-1 if i is out of range).  tsqr_profile_only(names) limits the recording
 * to the phases named in the comma-separated list `names` (NULL: every phase), so that a
 * timed run carries only the events it needs.  Process-wide; not meant for concurrent use. */
int tsqr_profile_start(void);
int tsqr_profile_stop(void);
int tsqr_profile_record(int i, const char** name, double* ms);
int tsqr_profile_only(const char* name);

/* Library identification string (static storage). */
const char* tsqr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TSQR_H */
