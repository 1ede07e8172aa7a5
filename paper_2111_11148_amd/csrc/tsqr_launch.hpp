// Host-side launchers of the libtsqr kernels (internal; the public interface is
// include/tsqr.h).  Every launcher enqueues on `stream` and returns hipError_t.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/tsqr.h"

namespace tsqr {

// ---- tiled partial-sum geometry -----------------------------------------------------
// Sketch partials: one (ceil(s/16) x ceil(n/16)) grid of 16x16 tiles per row block,
// stored tile-natively (tile, lane, 4 registers) in FP64.
struct SketchPlan {
  int it_total, jt_total;  // 16-row tiles of B, 16-column tiles of B
  int IT, JT, NW;          // i-tiles per wave, j-tiles per workgroup, waves per workgroup
  int igroups, jgroups;    // workgroup grid in the i and j directions
  int64_t rows_per_block;  // rows of A per workgroup (multiple of 32)
  int kblocks;             // number of row blocks
  size_t part_doubles;     // kblocks * it_total * jt_total * 256
};
SketchPlan plan_sketch(int64_t m, int n, int s);

struct GramPlan {
  int jt_total;  // 16-column tiles
  int ntiles;    // upper-triangular tiles (jt_total*(jt_total+1)/2)
  int64_t rows_per_block;
  int kblocks;
  size_t part_doubles;
  int wide;      // n > 256: 128-column block pairs (npairs of them), 64 tiles each
  int npairs;
};
GramPlan plan_gram(int64_t m, int n);

// ---- launchers ----------------------------------------------------------------------
// The launchers that take `gate` (a device int, or null) enqueue kernels that return at
// once when *gate == 0: a chain can then decide on the device whether a step runs, with
// no host wait, and stays capturable in a graph.
hipError_t launch_sketch(const SketchPlan& p, int64_t m, int n, const double* A, int64_t lda,
                         int s, uint64_t seed, double* part, hipStream_t st);
// B(s x n, ld ldb) = scale * sum of the sketch partials
hipError_t launch_sketch_reduce(const SketchPlan& p, int s, int n, const double* part,
                                double scale, double* B, int64_t ldb, hipStream_t st);
hipError_t launch_gram(const GramPlan& p, int64_t m, int n, const double* X, int64_t ldx,
                       double* part, hipStream_t st, const int* gate = nullptr);
// W(n x n, ld ldw, both triangles) = sum of the Gram partials
hipError_t launch_gram_reduce(const GramPlan& p, int n, const double* part, double* W,
                              int64_t ldw, hipStream_t st, const int* gate = nullptr);
// X = Y T^{-1} (T upper n x n); X may alias Y; `scratch` holds trsm_scratch_doubles(n)
size_t trsm_scratch_doubles(int n);
hipError_t launch_trsm(int64_t m, int n, const double* Y, int64_t ldy, const double* T,
                       int64_t ldt, double* X, int64_t ldx, double* scratch, hipStream_t st,
                       const int* gate = nullptr);
// the same in two steps: operand preparation (k_trsm_prep), then the solve
hipError_t launch_trsm_prepare(int n, const double* T, int64_t ldt, double* scratch,
                               hipStream_t st, const int* gate = nullptr);
hipError_t launch_trsm_solve(int64_t m, int n, const double* Y, int64_t ldy, const double* T,
                             int64_t ldt, double* X, int64_t ldx, double* scratch,
                             hipStream_t st, const int* gate = nullptr);
// R0 from the s x n sketch: Householder (variant 0) or partial-pivot LU (variant 1);
// `scratch` holds sketch_factor_scratch_doubles(s, n) doubles.
size_t sketch_factor_scratch_doubles(int s, int n);
hipError_t launch_sketch_factor(int variant, int s, int n, const double* B, int64_t ldb,
                                double* R, int64_t ldr, int* info, double* scratch,
                                hipStream_t st);
// Cholesky of the symmetric W (both triangles stored) into upper R; info stage
hipError_t launch_potrf(int n, const double* W, int64_t ldw, double* R, int64_t ldr, int stage,
                        int* info, double* scratch, hipStream_t st, double shift = 0.0,
                        const int* gate = nullptr);
// C = A B for upper-triangular n x n matrices
hipError_t launch_trmm_upper(int n, const double* A, int64_t lda, const double* B, int64_t ldb,
                             double* C, int64_t ldc, hipStream_t st, const int* gate = nullptr);
// If *info != 0, fill Q (m x n) and R (n x n, optional) with NaN
hipError_t launch_poison(const int* info, int64_t m, int n, double* Q, int64_t ldq, double* R,
                         int64_t ldr, hipStream_t st);
hipError_t launch_sketch_rows(int64_t m, int n, const double* A, int64_t lda, int s,
                              uint64_t seed, double* B, int64_t ldb, hipStream_t st);
hipError_t launch_add_diag(int n, double* W, int64_t ldw, double coef, const double* scale,
                           hipStream_t st, const int* gate = nullptr);
hipError_t launch_gemv_t(int64_t m, int n, const double* X, int64_t ldx, const double* b,
                         double* part, double* c, hipStream_t st);
size_t gemv_part_doubles(int64_t m, int n);
hipError_t launch_lsq_solve(int n, const double* U, int64_t ldu, const double* R0, int64_t ldr,
                            const double* c, double* x, const int* info, hipStream_t st);
hipError_t launch_set_int(int* p, int v, hipStream_t st);
hipError_t launch_identity(int n, double* Y, hipStream_t st);
// C = *flag ? B : A B (upper n x n)
hipError_t launch_trmm_or_copy(const int* flag, int n, const double* A, int64_t lda,
                               const double* B, int64_t ldb, double* C, int64_t ldc,
                               hipStream_t st);
// *need = breakdown in lp_info/info or ||W - I||_F > thresh (one workgroup)
hipError_t launch_pass_decide(int n, const double* W, int64_t ldw, const int* lp_info,
                              const int* info, double thresh, int* need, double* dev_out,
                              hipStream_t st, const int* gate = nullptr);

// ---- decisions of the mixed-precision chain, taken on the device --------------------------
// Control words of one mixed-precision factorization (in its workspace).  gate[k] = 1 when
// FP64 pass k runs; every kernel of pass k is gated by it, so the automatic mode enqueues
// its largest number of passes and the unneeded ones return at once.
constexpr int kMaxMixedPasses = 3;
struct MixedCtl {
  int stage;                     // the low-precision A R0^{-1} / Gram / Cholesky stage runs
  int lp_info;                   // its Cholesky breakdown (-1 when the stage did not run)
  int gate[kMaxMixedPasses + 1];  // pass k runs
  int skip[kMaxMixedPasses];     // 1 - gate[k]: the R product of pass k is a copy
  int bd[kMaxMixedPasses];       // pass k's unshifted Cholesky broke down
  int shifted[kMaxMixedPasses];  // pass k retries with the shifted Cholesky
  int need[kMaxMixedPasses + 2]; // scratch of the deviation kernel
  int one;                       // constant 1
  int passes;                    // passes run
  double dev[kMaxMixedPasses][2];  // ||W - I||_F and ||W||_F of pass k's Gram matrix
  double norms[4];               // ||R0||_F at [1], ||R0^{-1}||_F at [3]
};
enum MixedOp {
  kCtlInit,       // fixed passes (arg): gates of the fixed schedule; 0: automatic
  kCtlStage,      // stage = ||R0||_F ||R0^{-1}||_F u_p <= 1 (u_p = arg2)
  kCtlPassBegin,  // pass k: bd[k] = 0, skip[k] = !gate[k]
  kCtlShift,      // pass k: shifted[k] = gate[k] && bd[k]
  kCtlNext,       // pass k: gate[k+1] = gate[k] && (shifted[k] || dev[k][0] > arg2), k+1 < max
  kCtlEnd         // passes = sum of gates; *info = 5000 when the last allowed pass needed
                  // the shifted retry (the pass budget ran out); d_report = {passes, stage}
};
hipError_t launch_mixed_ctl(int op, int k, int arg, double arg2, MixedCtl* c, int* info,
                            int* d_passes, hipStream_t st);

// ---- low-precision phases (precision codes TSQR_LOWP_FP32 / TSQR_LOWP_BF16) -------------
size_t lowp_elem_bytes(int prec);
size_t rinv_lowp_bytes(int prec, int n);
hipError_t launch_sketch_lowp(int prec, const SketchPlan& p, int64_t m, int n, const double* A,
                              int64_t lda, uint64_t seed, double* part, hipStream_t st);
hipError_t launch_rinv_prep(int prec, int n, const double* Rinv, int64_t ldr, void* out,
                            hipStream_t st, const int* gate = nullptr);
hipError_t launch_apply_rinv_lowp(int prec, int64_t m, int n, const double* Y, int64_t ldy,
                                  const void* Ri, void* X, int64_t ldx, hipStream_t st,
                                  const int* gate = nullptr);
hipError_t launch_gram_lowp(int prec, const GramPlan& p, int64_t m, int n, const void* X,
                            int64_t ldx, double* part, hipStream_t st, const int* gate = nullptr);

// ---- batched factorizations -------------------------------------------------------------
// One problem of a batch as the batched kernels see it (device copy in the workspace).
struct BProb {
  const double* A;  // caller's input (m x n, ld lda)
  double* Q;        // caller's output (ld ldq)
  double* R;        // caller's output (ld ldr) or null
  int64_t m, lda, ldq, ldr;
  int n, s;
  uint32_t k0, k1;  // sketch seed halves
  double scale;     // 1 / sqrt(s)
  double* B;        // s x n sketch (ld s)
  double* R0;       // n x n factors (ld n)
  double* R1;
  double* R2;
  double* R10;
  double* W;        // Gram matrix (ld n)
  double* P;        // prepared triangular-solve tiles
  double* part;     // split-K partial sums
  int* info;
  int64_t sk_rpb;   // sketch: rows per block, row blocks, tile counts
  int sk_kblocks, sk_it, sk_jt;
  int gr_kblocks;   // Gram: row blocks, tiles
  int64_t gr_rpb;
  int gr_ntiles;
  int trsm_wgs;     // workgroups of each triangular solve
  int poison_wgs;
  int pad;
  // persistent schedule (one launch for the batch)
  int jt;                // 16-column tiles, rounded up to a power of two (<= 8)
  int qr_rpl, qr_cpw;    // register factorization of the sketch (rows, columns per lane)
  int po_rpl, po_cpw;    // register Cholesky
  int p_igroups;         // sketch i-groups per row block (groups of 16 row tiles of B)
  int p_jgroups;         // sketch column groups per row block (low precision: 4 tiles)
  int p_nsk;             // sketch tasks
  int p_ntrsm;           // tasks of each solve
  int* cnt;              // dependency counters, kPsSlots of them
};
// Dependency counters of a problem in the persistent schedule: tasks completed per step,
// and flags raised once a factor and its solve operands are ready.
enum PersistSlot {
  kPsSketch, kPsR0, kPsTrsm0, kPsGram1, kPsR1, kPsTrsm1, kPsGram2, kPsR2, kPsTrsm2, kPsSlots
};
// One workgroup's share: problem index and block coordinates.
struct BItem {
  int pid, x, y, z;
};

hipError_t launch_b_sketch_lowp(int prec, int IT, int JT, int NW, const BItem* items, int nitems,
                                const BProb* probs, hipStream_t st);
hipError_t launch_b_sketch(int IT, int JT, int NW, const BItem* items, int nitems,
                           const BProb* probs, hipStream_t st);
hipError_t launch_b_sketch_reduce(const BItem* items, int nitems, const BProb* probs,
                                  hipStream_t st);
// variant 0: Householder QR, 1: LU (register kernels, s <= 512, n <= 128)
hipError_t launch_b_factor(int variant, int RPL, int CPW, const BItem* items, int nitems,
                           const BProb* probs, hipStream_t st);
// which: 0 = R0, 1 = R1, 2 = R2
hipError_t launch_b_trsm_prep(int which, const BItem* items, int nitems, const BProb* probs,
                              hipStream_t st);
// src: 0 = A (lda), 1 = Q (ldq); X = Q
hipError_t launch_b_trsm(int JT, int src, const BItem* items, int nitems, const BProb* probs,
                         hipStream_t st);
hipError_t launch_b_gram(int JT, const BItem* items, int nitems, const BProb* probs,
                         hipStream_t st);
hipError_t launch_b_gram_reduce(const BItem* items, int nitems, const BProb* probs,
                                hipStream_t st);
// which: 1 = R1, 2 = R2
hipError_t launch_b_potrf(int RPL, int CPW, int which, int stage, const BItem* items,
                          int nitems, const BProb* probs, hipStream_t st);
// which: 0 = R10 = R1 R0, 1 = R = R2 R10 (problems without R skip)
hipError_t launch_b_trmm(int which, const BItem* items, int nitems, const BProb* probs,
                         hipStream_t st);
hipError_t launch_b_poison(const BItem* items, int nitems, const BProb* probs, hipStream_t st);
hipError_t launch_b_set_info(const BItem* items, int nitems, const BProb* probs, hipStream_t st);
// The whole batch in one persistent launch (after a kernel that clears its counters).
size_t persistent_lds_bytes(int max_jt, int max_rpl_cpw, int precision);
// stats: null, or 18 device counters of wall-clock ticks per task kind (wait, body,
// finishing step)
hipError_t launch_b_persistent(int variant, int precision, const BProb* probs, int nprobs,
                               const int4* tasks, int ntasks, int* ctl, size_t lds_bytes,
                               unsigned long long* stats, hipStream_t st);

// ---- accuracy metrics (double-double) and attainable-peak probes -------------------------
size_t metrics_workspace_bytes(int64_t m, int n);
// out[0] = ||Q^T Q - I||_F; out[1] = ||A - Q R||_F / ||A||_F (NaN when A or R is null)
hipError_t launch_metrics(int64_t m, int n, const double* A, int64_t lda, const double* Q,
                          int64_t ldq, const double* R, int64_t ldr, double* out, void* work,
                          hipStream_t st);
hipError_t launch_probe_stream(int kind, const void* src, void* dst, size_t bytes,
                               int wgs_per_cu, int unroll, int nontemporal, double* sink,
                               hipStream_t st);
hipError_t launch_probe_mfma(int kind, int waves_per_simd, int chains, int64_t iters,
                             double* sink, double* flops, hipStream_t st);

// ---- test / debug kernels -------------------------------------------------------------
hipError_t launch_philox_words(int64_t count, const uint32_t* ctr, uint64_t seed, uint32_t* out,
                               hipStream_t st);
hipError_t launch_sketch_normals(uint64_t seed, int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                                 double* Z, int64_t ldz, hipStream_t st);

int device_cu_count();

}  // namespace tsqr
