// C ABI of libtsqr (declared in include/tsqr.h): argument validation, workspace layout
// and the stream-ordered sequence of kernels of randomized XR-preconditioned CholeskyQR.
#include <math.h>
#include <string.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tsqr.h"
#include "tsqr_launch.hpp"

namespace tsqr {

int device_cu_count() {
  static std::mutex mu;
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> g(mu);
  if (!cache[dev]) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cache[dev] = cus;
  }
  return cache[dev];
}

namespace {

constexpr int64_t kMaxSketchRows = 8192;
constexpr int64_t kMaxN = 1024;     // widest n of the FP64 path
constexpr int64_t kMaxNLowp = 256;  // widest n of the low-precision kernels
// u of the suggested sCholeskyQR3 shift 11 (m n + n (n + 1)) u ||A||_2^2 (paper Section 2.1):
// the machine precision 2^-52 the paper defines for double precision (Section 4.1)
constexpr double kMachEps = 0x1p-52;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t info, B, R0, R1, R2, R10, W, fac, Tt, part, total;
  SketchPlan sp;
  GramPlan gp;
};

Layout make_layout(int64_t m, int64_t n, int64_t s) {
  Layout L{};
  L.sp = plan_sketch(m, (int)n, (int)s);
  L.gp = plan_gram(m, (int)n);
  const size_t nn = (size_t)n * n * sizeof(double);
  size_t off = 0;
  L.info = off; off += 256;
  L.B = off; off += align256((size_t)s * n * sizeof(double));
  L.R0 = off; off += align256(nn);
  L.R1 = off; off += align256(nn);
  L.R2 = off; off += align256(nn);
  L.R10 = off; off += align256(nn);
  L.W = off; off += align256(nn);
  {
    const size_t f = sketch_factor_scratch_doubles((int)s, (int)n);
    const size_t nn2 = (size_t)n * n;
    L.fac = off;
    off += align256((f > nn2 ? f : nn2) * sizeof(double));
  }
  L.Tt = off; off += align256(trsm_scratch_doubles((int)n) * sizeof(double));
  L.part = off;
  const size_t part = L.sp.part_doubles > L.gp.part_doubles ? L.sp.part_doubles : L.gp.part_doubles;
  off += align256(part * sizeof(double));
  L.total = off;
  return L;
}

inline bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + bbytes && pb < pa + abytes;
}

inline size_t span_bytes(int64_t rows, int64_t cols, int64_t ld) {
  return ((size_t)(cols - 1) * (size_t)ld + (size_t)rows) * sizeof(double);
}

#define TSQR_CHECK(expr)                   \
  do {                                     \
    if ((expr) != hipSuccess) return TSQR_ERR_HIP; \
  } while (0)

// ---- phase timing: HIP events recorded on the caller's stream around each launch ----
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_live;
std::vector<std::pair<const char*, double>> g_prof_done;
std::vector<hipEvent_t> g_prof_pool;
std::string g_prof_only;  // empty: every phase

// g_prof_only: empty, or a comma-separated list of phase names
bool prof_on(const char* name) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (!g_prof_on) return false;
  if (g_prof_only.empty()) return true;
  const size_t len = strlen(name);
  size_t pos = 0;
  while (pos <= g_prof_only.size()) {
    size_t end = g_prof_only.find(',', pos);
    if (end == std::string::npos) end = g_prof_only.size();
    if (end - pos == len && g_prof_only.compare(pos, len, name) == 0) return true;
    pos = end + 1;
  }
  return false;
}

void prof_release(hipEvent_t e) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_pool.push_back(e);
}

hipEvent_t prof_event() {
  std::lock_guard<std::mutex> g(g_prof_mu);
  hipEvent_t e = nullptr;
  if (!g_prof_pool.empty()) {
    e = g_prof_pool.back();
    g_prof_pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

void prof_push(const char* name, hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_live.push_back(ProfRec{name, a, b});
}

#define TSQR_PHASE(name, expr)                                               \
  do {                                                                       \
    hipEvent_t ev_a_ = nullptr, ev_b_ = nullptr;                             \
    const bool on_ = prof_on(name);                                          \
    if (on_ && (ev_a_ = prof_event())) (void)hipEventRecord(ev_a_, st);      \
    const hipError_t err_ = (expr);                                          \
    if (on_ && ev_a_) {                                                      \
      if ((ev_b_ = prof_event())) {                                          \
        (void)hipEventRecord(ev_b_, st);                                     \
        prof_push(name, ev_a_, ev_b_);                                       \
      } else {                                                               \
        prof_release(ev_a_);                                                 \
      }                                                                      \
    }                                                                        \
    if (err_ != hipSuccess) return TSQR_ERR_HIP;                             \
  } while (0)

// sketch_kind 0: Gaussian B = S A; 1: row extraction B = A(rows, :).
int run_chain(int variant, int64_t m, int64_t n, const double* A, int64_t lda, int64_t s,
              uint64_t seed, int extra_pass, double* Q, int64_t ldq, double* R, int64_t ldr,
              void* work, int* d_info, hipStream_t st, int sketch_kind = 0) {
  const Layout L = make_layout(m, n, s);
  char* base = (char*)work;
  int* info = d_info ? d_info : (int*)(base + L.info);
  double* B = (double*)(base + L.B);
  double* R0 = (double*)(base + L.R0);
  double* R1 = (double*)(base + L.R1);
  double* R2 = (double*)(base + L.R2);
  double* R10 = (double*)(base + L.R10);
  double* W = (double*)(base + L.W);
  double* fac = (double*)(base + L.fac);
  double* Tt = (double*)(base + L.Tt);
  double* part = (double*)(base + L.part);
  const int ni = (int)n, si = (int)s;

  TSQR_CHECK(launch_set_int(info, 0, st));
  if (sketch_kind == 1) {
    // B = P A, s sampled rows  (paper Section 2.3, row extraction)
    TSQR_PHASE("sketch_rows", launch_sketch_rows(m, ni, A, lda, si, seed, B, s, st));
  } else {
    // B = S A  (paper Section 2.3, Gaussian ensemble)
    TSQR_PHASE("sketch", launch_sketch(L.sp, m, ni, A, lda, si, seed, part, st));
    TSQR_PHASE("sketch_reduce",
               launch_sketch_reduce(L.sp, si, ni, part, 1.0 / sqrt((double)s), B, s, st));
  }
  // R0 = R factor of B
  TSQR_PHASE(variant == 1 ? "sketch_lu" : "sketch_qr",
             launch_sketch_factor(variant, si, ni, B, s, R0, n, info, fac, st));
  // A1 = A R0^{-1} (into Q), W1 = A1^T A1, R1 = chol(W1), Q1 = A1 R1^{-1}
  TSQR_PHASE("trsm_prep_r0", launch_trsm_prepare(ni, R0, n, Tt, st));
  TSQR_PHASE("trsm_r0", launch_trsm_solve(m, ni, A, lda, R0, n, Q, ldq, Tt, st));
  TSQR_PHASE("gram1", launch_gram(L.gp, m, ni, Q, ldq, part, st));
  TSQR_PHASE("gram1_reduce", launch_gram_reduce(L.gp, ni, part, W, n, st));
  TSQR_PHASE("potrf1", launch_potrf(ni, W, n, R1, n, 2, info, fac, st));
  TSQR_PHASE("trsm_prep_r1", launch_trsm_prepare(ni, R1, n, Tt, st));
  TSQR_PHASE("trsm_r1", launch_trsm_solve(m, ni, Q, ldq, R1, n, Q, ldq, Tt, st));
  if (extra_pass) {
    // W2 = Q1^T Q1, R2 = chol(W2), Q = Q1 R2^{-1}
    TSQR_PHASE("gram2", launch_gram(L.gp, m, ni, Q, ldq, part, st));
    TSQR_PHASE("gram2_reduce", launch_gram_reduce(L.gp, ni, part, W, n, st));
    TSQR_PHASE("potrf2", launch_potrf(ni, W, n, R2, n, 3, info, fac, st));
    TSQR_PHASE("trsm_prep_r2", launch_trsm_prepare(ni, R2, n, Tt, st));
    TSQR_PHASE("trsm_r2", launch_trsm_solve(m, ni, Q, ldq, R2, n, Q, ldq, Tt, st));
  }
  if (R) {
    if (extra_pass) {
      TSQR_PHASE("trmm", launch_trmm_upper(ni, R1, n, R0, n, R10, n, st));
      TSQR_PHASE("trmm", launch_trmm_upper(ni, R2, n, R10, n, R, ldr, st));
    } else {
      TSQR_PHASE("trmm", launch_trmm_upper(ni, R1, n, R0, n, R, ldr, st));
    }
  }
  TSQR_PHASE("poison", launch_poison(info, m, ni, Q, ldq, R, ldr, st));
  return TSQR_OK;
}

// Validation shared by the plain and workspace forms; returns 0 or the code of the first
// invalid argument expressed in the plain form's numbering (caller remaps).
enum ArgErr { E_OK = 0, E_M, E_N, E_A, E_LDA, E_S, E_Q, E_LDQ, E_R, E_LDR };

ArgErr validate(int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, const double* Q,
                int64_t ldq, const double* R, int64_t ldr) {
  if (n < 1) return E_N;
  if (m < 1 || m < n) return E_M;
  if (!A) return E_A;
  if (lda < m) return E_LDA;
  if (s < n || s > kMaxSketchRows) return E_S;
  if (!Q) return E_Q;
  if (ldq < m) return E_LDQ;
  if (overlaps(A, span_bytes(m, n, lda), Q, span_bytes(m, n, ldq))) return E_Q;
  if (R) {
    if (ldr < n) return E_LDR;
    if (overlaps(R, span_bytes(n, n, ldr), Q, span_bytes(m, n, ldq)) ||
        overlaps(R, span_bytes(n, n, ldr), A, span_bytes(m, n, lda)))
      return E_R;
  }
  return E_OK;
}

int plain_form(int variant, int64_t m, int64_t n, const double* A, int64_t lda, int64_t s,
               uint64_t seed, double* Q, double* R, void* stream) {
  const ArgErr e = validate(m, n, A, lda, s, Q, m, R, n);
  switch (e) {
    case E_OK: break;
    case E_M: return -1;
    case E_N: return -2;
    case E_A: return -3;
    case E_LDA: return -4;
    case E_S: return -5;
    case E_Q: case E_LDQ: return -7;
    case E_R: case E_LDR: return -8;
  }
  if (n > kMaxN) return TSQR_ERR_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = make_layout(m, n, s).total;
  void* work = nullptr;
  if (hipMallocAsync(&work, bytes, st) != hipSuccess) return TSQR_ERR_HIP;
  const int rc = run_chain(variant, m, n, A, lda, s, seed, 1, Q, m, R, n, work, nullptr, st);
  if (hipFreeAsync(work, st) != hipSuccess && rc == TSQR_OK) return TSQR_ERR_HIP;
  return rc;
}

// ---- CholeskyQR, CholeskyQR2, shifted CholeskyQR3 (paper Section 2.1) -----------------
struct CholLayout {
  size_t info, W, Rk, Racc, Rt, fac, Tt, part, dev, need, total;
  GramPlan gp;
};

CholLayout make_chol_layout(int64_t m, int64_t n) {
  CholLayout L{};
  L.gp = plan_gram(m, (int)n);
  const size_t nn = align256((size_t)n * n * sizeof(double));
  size_t off = 0;
  L.info = off; off += 256;
  L.W = off; off += nn;
  L.Rk = off; off += nn;
  L.Racc = off; off += nn;
  L.Rt = off; off += nn;
  L.fac = off; off += nn;
  L.Tt = off; off += align256(trsm_scratch_doubles((int)n) * sizeof(double));
  L.part = off; off += align256(L.gp.part_doubles * sizeof(double));
  L.dev = off; off += 256;
  L.need = off; off += 256;
  L.total = off;
  return L;
}

// Passes k = 1..npass: W = X^T X (X = A, then Q), on the first pass plus the shift when
// shifted, Rk = chol(W) (stage k), Q = X Rk^{-1}, R = Rk ... R1.  Shift: >= 0 absolute,
// < 0 the suggested 11 (m n + n (n+1)) u ||A||_2^2 with ||A||_2^2 <= ||A^T A||_F taken on
// the device.
int run_cholqr(int npass, bool shifted, int64_t m, int64_t n, const double* A, int64_t lda,
               double shift, double* Q, int64_t ldq, double* R, int64_t ldr, void* work,
               int* d_info, hipStream_t st) {
  const CholLayout L = make_chol_layout(m, n);
  char* base = (char*)work;
  int* info = d_info ? d_info : (int*)(base + L.info);
  double* W = (double*)(base + L.W);
  double* Rk = (double*)(base + L.Rk);
  double* Racc = (double*)(base + L.Racc);
  double* Rt = (double*)(base + L.Rt);
  double* fac = (double*)(base + L.fac);
  double* Tt = (double*)(base + L.Tt);
  double* part = (double*)(base + L.part);
  double* dev = (double*)(base + L.dev);
  int* need = (int*)(base + L.need);
  const int ni = (int)n;
  TSQR_CHECK(launch_set_int(info, 0, st));
  for (int pass = 0; pass < npass; ++pass) {
    const double* X = pass == 0 ? A : Q;
    const int64_t ldxx = pass == 0 ? lda : ldq;
    TSQR_PHASE("gram", launch_gram(L.gp, m, ni, X, ldxx, part, st));
    TSQR_PHASE("gram_reduce", launch_gram_reduce(L.gp, ni, part, W, n, st));
    if (pass == 0 && shifted) {
      if (shift < 0.0) {
        const double c = 11.0 * ((double)m * (double)n + (double)n * (double)(n + 1)) * kMachEps;
        TSQR_CHECK(launch_pass_decide(ni, W, n, nullptr, nullptr, 0.0, need, dev, st));
        TSQR_PHASE("shift", launch_add_diag(ni, W, n, c, dev + 1, st));  // dev[1] = ||W||_F
      } else {
        TSQR_PHASE("shift", launch_add_diag(ni, W, n, shift, nullptr, st));
      }
    }
    TSQR_PHASE("potrf", launch_potrf(ni, W, n, pass == 0 ? Racc : Rk, n, pass + 1, info, fac, st));
    TSQR_PHASE("trsm", launch_trsm(m, ni, X, ldxx, pass == 0 ? Racc : Rk, n, Q, ldq, Tt, st));
    if (pass > 0) {
      TSQR_PHASE("trmm", launch_trmm_upper(ni, Rk, n, Racc, n, Rt, n, st));
      std::swap(Racc, Rt);
    }
  }
  if (R) TSQR_CHECK(hipMemcpy2DAsync(R, ldr * sizeof(double), Racc, n * sizeof(double),
                                     n * sizeof(double), n, hipMemcpyDeviceToDevice, st));
  TSQR_PHASE("poison", launch_poison(info, m, ni, Q, ldq, R, ldr, st));
  return TSQR_OK;
}

// ---- least squares preconditioned by the sketch's R (paper Section 5.2) -----------------
struct LsqLayout {
  Layout base;
  size_t Bm, cpart, c, total;
};

LsqLayout make_lsq_layout(int64_t m, int64_t n, int64_t s) {
  LsqLayout L{};
  L.base = make_layout(m, n, s);
  size_t off = L.base.total;
  L.Bm = off; off += align256((size_t)m * n * sizeof(double));
  L.cpart = off; off += align256(gemv_part_doubles(m, (int)n) * sizeof(double));
  L.c = off; off += align256((size_t)n * sizeof(double));
  L.total = off;
  return L;
}

// R0 from the sketch; B = A R0^{-1}; G = B^T B = U^T U (stage 2); c = B^T b; then
// U^T z = c, U y = z, R0 x = y.
int run_lstsq(int variant, int sketch_kind, int64_t m, int64_t n, const double* A, int64_t lda,
              const double* b, int64_t s, uint64_t seed, double* x, void* work, int* d_info,
              hipStream_t st) {
  const LsqLayout M = make_lsq_layout(m, n, s);
  const Layout& L = M.base;
  char* base = (char*)work;
  int* info = d_info ? d_info : (int*)(base + L.info);
  double* Bs = (double*)(base + L.B);
  double* R0 = (double*)(base + L.R0);
  double* U = (double*)(base + L.R1);
  double* G = (double*)(base + L.W);
  double* fac = (double*)(base + L.fac);
  double* Tt = (double*)(base + L.Tt);
  double* part = (double*)(base + L.part);
  double* Bm = (double*)(base + M.Bm);
  double* cpart = (double*)(base + M.cpart);
  double* c = (double*)(base + M.c);
  const int ni = (int)n, si = (int)s;
  TSQR_CHECK(launch_set_int(info, 0, st));
  if (sketch_kind == 1) {
    TSQR_PHASE("sketch_rows", launch_sketch_rows(m, ni, A, lda, si, seed, Bs, s, st));
  } else {
    TSQR_PHASE("sketch", launch_sketch(L.sp, m, ni, A, lda, si, seed, part, st));
    TSQR_PHASE("sketch_reduce",
               launch_sketch_reduce(L.sp, si, ni, part, 1.0 / sqrt((double)s), Bs, s, st));
  }
  TSQR_PHASE(variant == 1 ? "sketch_lu" : "sketch_qr",
             launch_sketch_factor(variant, si, ni, Bs, s, R0, n, info, fac, st));
  TSQR_PHASE("trsm_r0", launch_trsm(m, ni, A, lda, R0, n, Bm, m, Tt, st));
  TSQR_PHASE("gram", launch_gram(L.gp, m, ni, Bm, m, part, st));
  TSQR_PHASE("gram_reduce", launch_gram_reduce(L.gp, ni, part, G, n, st));
  TSQR_PHASE("gemv", launch_gemv_t(m, ni, Bm, m, b, cpart, c, st));
  TSQR_PHASE("potrf", launch_potrf(ni, G, n, U, n, 2, info, fac, st));
  TSQR_PHASE("solve", launch_lsq_solve(ni, U, n, R0, n, c, x, info, st));
  return TSQR_OK;
}

// ---- mixed precision ---------------------------------------------------------------
// The input type `lowp` is that of the sketch's matrix cores.  The preconditioning stage
// after it (A1 = A R0^{-1}, its Gram matrix) takes FP32 inputs for either type: with BF16
// inputs it could only save an FP64 pass below cond(A) ~ 1e2.
constexpr int kStagePrec = TSQR_LOWP_FP32;

// Extra workspace after the FP64 layout: A1 in the stage's type, R0^{-1} (FP64 and
// rounded), identity, R01 = R1 R0, two more n x n factors and the chain's control words.
struct MixedLayout {
  Layout base;
  size_t A1, Rinv, Ri_lp, Id, R01, R3, Rt, ctl, total;
};

MixedLayout make_mixed_layout(int64_t m, int64_t n, int64_t s, int lowp) {
  MixedLayout L{};
  L.base = make_layout(m, n, s);
  const size_t nn = (size_t)n * n * sizeof(double);
  size_t off = L.base.total;
  (void)lowp;  // the sketch needs no workspace of its own type
  L.A1 = off; off += align256((size_t)m * n * lowp_elem_bytes(kStagePrec));
  L.Rinv = off; off += align256(nn);
  L.Ri_lp = off; off += align256(rinv_lowp_bytes(kStagePrec, (int)n));
  L.Id = off; off += align256(nn);
  L.R01 = off; off += align256(nn);
  L.R3 = off; off += align256(nn);
  L.Rt = off; off += align256(nn);
  L.ctl = off; off += align256(sizeof(MixedCtl));
  L.total = off;
  return L;
}

// Deviation of Q1^T Q1 from I above which another FP64 CholeskyQR pass is run in the
// automatic mode: ||W - I||_F <= 1/2 gives cond(W) <= 3, i.e. cond(Q1) <= 1.8.
constexpr double kPassThresh = 0.5;

// Automatic mode: the low-precision stage (A1 = A R0^{-1}, its Gram matrix and Cholesky)
// runs only when ||R0||_F ||R0^{-1}||_F u_p <= 1, an upper bound of cond(R0) u_p with u_p
// the stage's FP32 unit 2^-24: then the rounding of A to FP32 perturbs A R0^{-1} by well
// under one and the stage can leave a single FP64 pass. Otherwise it could not save a
// pass, and the FP64 passes start from A R0^{-1} (low precision for the sketch only).
constexpr double kStageUnit = 0x1p-24;

int run_chain_mixed(int variant, int lowp, int64_t m, int64_t n, const double* A, int64_t lda,
                    int64_t s, uint64_t seed, int fp64_passes, double* Q, int64_t ldq,
                    double* R, int64_t ldr, void* work, int* d_info, int* d_report,
                    hipStream_t st) {
  const MixedLayout M = make_mixed_layout(m, n, s, lowp);
  const Layout& L = M.base;
  char* base = (char*)work;
  int* info = d_info ? d_info : (int*)(base + L.info);
  double* B = (double*)(base + L.B);
  double* R0 = (double*)(base + L.R0);
  double* R1 = (double*)(base + L.R1);
  double* R2 = (double*)(base + L.R2);
  double* Racc = (double*)(base + L.R10);
  double* W = (double*)(base + L.W);
  double* fac = (double*)(base + L.fac);
  double* Tt = (double*)(base + L.Tt);
  double* part = (double*)(base + L.part);
  void* A1 = base + M.A1;
  double* Rinv = (double*)(base + M.Rinv);
  void* Ri_lp = base + M.Ri_lp;
  double* Id = (double*)(base + M.Id);
  double* R01 = (double*)(base + M.R01);
  double* R3 = (double*)(base + M.R3);
  double* Rt = (double*)(base + M.Rt);
  MixedCtl* c = (MixedCtl*)(base + M.ctl);
  const int ni = (int)n, si = (int)s;
  const bool automatic = fp64_passes == 0;
  const int max_passes = automatic ? kMaxMixedPasses : fp64_passes;

  TSQR_CHECK(launch_set_int(info, 0, st));
  TSQR_CHECK(launch_mixed_ctl(kCtlInit, 0, fp64_passes, 0.0, c, info, nullptr, st));
  // low-precision sketch, FP64 factor of the sketch, FP64 inverse
  TSQR_PHASE("sketch_lowp", launch_sketch_lowp(lowp, L.sp, m, ni, A, lda, seed, part, st));
  TSQR_PHASE("sketch_reduce",
             launch_sketch_reduce(L.sp, si, ni, part, 1.0 / sqrt((double)s), B, s, st));
  TSQR_PHASE(variant == 1 ? "sketch_lu" : "sketch_qr",
             launch_sketch_factor(variant, si, ni, B, s, R0, n, info, fac, st));
  TSQR_CHECK(launch_identity(ni, Id, st));
  TSQR_PHASE("trtri_r0", launch_trsm(n, ni, Id, n, R0, n, Rinv, n, Tt, st));
  if (automatic) {
    // ||R0||_F and ||R0^{-1}||_F on the device, then the stage decision (R12)
    TSQR_CHECK(launch_pass_decide(ni, R0, n, nullptr, nullptr, 0.0, c->need + 3, c->norms, st));
    TSQR_CHECK(launch_pass_decide(ni, Rinv, n, nullptr, nullptr, 0.0, c->need + 4, c->norms + 2,
                                  st));
    TSQR_CHECK(launch_mixed_ctl(kCtlStage, 0, 0, kStageUnit, c, info, nullptr, st));
  }
  // low-precision preconditioner apply, first Gram matrix and its Cholesky factor (gated:
  // in the automatic mode they return at once when the stage is not worth running)
  const int* sg = &c->stage;
  TSQR_PHASE("rinv_round", launch_rinv_prep(kStagePrec, ni, Rinv, n, Ri_lp, st, sg));
  TSQR_PHASE("apply_lowp",
             launch_apply_rinv_lowp(kStagePrec, m, ni, A, lda, Ri_lp, A1, m, st, sg));
  TSQR_PHASE("gram_lowp", launch_gram_lowp(kStagePrec, L.gp, m, ni, A1, m, part, st, sg));
  TSQR_PHASE("gram1_reduce", launch_gram_reduce(L.gp, ni, part, W, n, st, sg));
  TSQR_PHASE("potrf1", launch_potrf(ni, W, n, R1, n, 2, &c->lp_info, fac, st, 0.0, sg));
  // R01 = R1 R0, or R0 alone when the low-precision Cholesky broke down or did not run
  TSQR_PHASE("trmm", launch_trmm_or_copy(&c->lp_info, ni, R1, n, R0, n, R01, n, st));
  // FP64 CholeskyQR passes on A R01^{-1}, from the FP64 A
  TSQR_PHASE("trsm_r01", launch_trsm(m, ni, A, lda, R01, n, Q, ldq, Tt, st));
  // Pass k (gated by gate[k]): W = Q^T Q, Rk = chol(W), Q = Q Rk^{-1}, R = Rk R.  Fixed
  // mode: exactly fp64_passes passes.  Automatic mode: a breakdown is retried with the
  // shift 11 (m n + n (n + 1)) u ||W||_F on the diagonal (the shifted CholeskyQR of the
  // paper's Section 2.1), and pass k + 1 runs while pass k needed the shift or its input
  // deviated from orthonormality by more than the threshold.  Every decision is taken by
  // a one-thread kernel from device data; the host never waits.
  double* Rcur = R01;  // R accumulated so far
  for (int pass = 0; pass < max_passes; ++pass) {
    double* Rk = (pass == 0) ? R2 : R3;
    double* Rnext = (Rcur == Racc) ? Rt : Racc;
    const int stage = 3 + (pass > 0);
    const int* g = &c->gate[pass];
    TSQR_CHECK(launch_mixed_ctl(kCtlPassBegin, pass, 0, 0.0, c, info, nullptr, st));
    TSQR_PHASE("gram", launch_gram(L.gp, m, ni, Q, ldq, part, st, g));
    TSQR_PHASE("gram_reduce", launch_gram_reduce(L.gp, ni, part, W, n, st, g));
    if (automatic) {
      TSQR_CHECK(launch_pass_decide(ni, W, n, nullptr, nullptr, kPassThresh, c->need + pass,
                                    c->dev[pass], st, g));
      TSQR_PHASE("potrf", launch_potrf(ni, W, n, Rk, n, stage, &c->bd[pass], fac, st, 0.0, g));
      TSQR_CHECK(launch_mixed_ctl(kCtlShift, pass, 0, 0.0, c, info, nullptr, st));
      const double coef = 11.0 * ((double)m * (double)n + (double)n * (double)(n + 1)) * kMachEps;
      const int* sh = &c->shifted[pass];
      TSQR_CHECK(launch_add_diag(ni, W, n, coef, &c->dev[pass][1], st, sh));
      TSQR_PHASE("potrf_shifted", launch_potrf(ni, W, n, Rk, n, stage, info, fac, st, 0.0, sh));
    } else {
      TSQR_PHASE("potrf", launch_potrf(ni, W, n, Rk, n, stage, info, fac, st, 0.0, g));
    }
    TSQR_PHASE("trsm", launch_trsm(m, ni, Q, ldq, Rk, n, Q, ldq, Tt, st, g));
    TSQR_PHASE("trmm", launch_trmm_or_copy(&c->skip[pass], ni, Rk, n, Rcur, n, Rnext, n, st));
    if (automatic)
      TSQR_CHECK(launch_mixed_ctl(kCtlNext, pass, max_passes, kPassThresh, c, info, nullptr, st));
    Rcur = Rnext;
  }
  TSQR_CHECK(
      launch_mixed_ctl(kCtlEnd, 0, automatic ? max_passes : 0, 0.0, c, info, d_report, st));
  if (R) TSQR_PHASE("trmm", launch_trmm_or_copy(&c->one, ni, Rcur, n, Rcur, n, R, ldr, st));
  TSQR_PHASE("poison", launch_poison(info, m, ni, Q, ldq, R, ldr, st));
  return TSQR_OK;
}

}  // namespace
}  // namespace tsqr

using namespace tsqr;

// ---- no-allocation entry point: the workspace lives in a device array of fixed size ----
// Each GPU that loads the library holds its own copy of `scratch` until the process ends.
// In host code the array's name is only a stand-in for the symbol; the device address is
// resolved once per device (with that device current) and kept.
static __device__ __align__(256) unsigned char scratch[TSQR_STATIC_SCRATCH_BYTES];

namespace tsqr {
namespace {
std::mutex g_scratch_mu;
void* g_scratch_addr[64] = {nullptr};

// Device address of this device's copy of `scratch`, or null on failure.
void* static_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch_addr[dev] = ptr;
  }
  return g_scratch_addr[dev];
}
}  // namespace
}  // namespace tsqr

extern "C" {

const char* tsqr_version(void) { return "libtsqr 0.1 (gfx950, FP64 MFMA)"; }

int tsqr_profile_start(void) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (auto& r : g_prof_live) {
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_live.clear();
  g_prof_done.clear();
  g_prof_on = true;
  return TSQR_OK;
}

int tsqr_profile_stop(void) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_on = false;
  g_prof_done.clear();
  int rc = TSQR_OK;
  for (auto& r : g_prof_live) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      rc = TSQR_ERR_HIP;
    g_prof_done.emplace_back(r.name, (double)ms);
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_live.clear();
  return rc == TSQR_OK ? (int)g_prof_done.size() : rc;
}

int tsqr_profile_only(const char* name) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_only = name ? name : "";
  return TSQR_OK;
}

int tsqr_profile_record(int i, const char** name, double* ms) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (i < 0 || i >= (int)g_prof_done.size()) return -1;
  if (name) *name = g_prof_done[i].first;
  if (ms) *ms = g_prof_done[i].second;
  return TSQR_OK;
}

int tsqr_rqr_cholqr(int64_t m, int64_t n, const double* A, int64_t lda, int64_t sketch_rows,
                    uint64_t seed, double* Q, double* R, void* stream) {
  return plain_form(TSQR_VARIANT_RQR, m, n, A, lda, sketch_rows, seed, Q, R, stream);
}

int tsqr_rlu_cholqr(int64_t m, int64_t n, const double* A, int64_t lda, int64_t sketch_rows,
                    uint64_t seed, double* Q, double* R, void* stream) {
  return plain_form(TSQR_VARIANT_RLU, m, n, A, lda, sketch_rows, seed, Q, R, stream);
}

size_t tsqr_workspace_bytes(int64_t m, int64_t n, int64_t sketch_rows) {
  if (n < 1 || m < n || sketch_rows < n || sketch_rows > kMaxSketchRows) return 0;
  return make_layout(m, n, sketch_rows).total;
}

int tsqr_rxr_cholqr_ws(int variant, int64_t m, int64_t n, const double* A, int64_t lda,
                       int64_t sketch_rows, uint64_t seed, int extra_pass, double* Q,
                       int64_t ldq, double* R, int64_t ldr, void* work, size_t work_bytes,
                       int* d_info, void* stream) {
  if (variant != TSQR_VARIANT_RQR && variant != TSQR_VARIANT_RLU) return -1;
  const ArgErr e = validate(m, n, A, lda, sketch_rows, Q, ldq, R, ldr);
  switch (e) {
    case E_OK: break;
    case E_M: return -2;
    case E_N: return -3;
    case E_A: return -4;
    case E_LDA: return -5;
    case E_S: return -6;
    case E_Q: return -9;
    case E_LDQ: return -10;
    case E_R: return -11;
    case E_LDR: return -12;
  }
  if (!work) return -13;
  if (n > kMaxN) return TSQR_ERR_UNSUPPORTED;
  if (work_bytes < make_layout(m, n, sketch_rows).total) return TSQR_ERR_WORKSPACE;
  return run_chain(variant, m, n, A, lda, sketch_rows, seed, extra_pass != 0, Q, ldq, R, ldr, work,
                   d_info, (hipStream_t)stream);
}

int tsqr_rxr_cholqr_noalloc(int variant, int64_t m, int64_t n, const double* A, int64_t lda,
                            int64_t sketch_rows, uint64_t seed, int extra_pass, double* Q,
                            int64_t ldq, double* R, int64_t ldr, int* d_info, void* stream) {
  if (variant != TSQR_VARIANT_RQR && variant != TSQR_VARIANT_RLU) return -1;
  const ArgErr e = validate(m, n, A, lda, sketch_rows, Q, ldq, R, ldr);
  switch (e) {
    case E_OK: break;
    case E_M: return -2;
    case E_N: return -3;
    case E_A: return -4;
    case E_LDA: return -5;
    case E_S: return -6;
    case E_Q: return -9;
    case E_LDQ: return -10;
    case E_R: return -11;
    case E_LDR: return -12;
  }
  if (n > kMaxN) return TSQR_ERR_UNSUPPORTED;
  if (make_layout(m, n, sketch_rows).total > (size_t)TSQR_STATIC_SCRATCH_BYTES)
    return TSQR_ERR_WORKSPACE;
  void* work = static_scratch();
  if (!work) return TSQR_ERR_HIP;
  return run_chain(variant, m, n, A, lda, sketch_rows, seed, extra_pass != 0, Q, ldq, R, ldr, work,
                   d_info, (hipStream_t)stream);
}

int tsqr_rxr_cholqr_rows_ws(int variant, int64_t m, int64_t n, const double* A, int64_t lda,
                            int64_t sketch_rows, uint64_t seed, int extra_pass, double* Q,
                            int64_t ldq, double* R, int64_t ldr, void* work, size_t work_bytes,
                            int* d_info, void* stream) {
  if (variant != TSQR_VARIANT_RQR && variant != TSQR_VARIANT_RLU) return -1;
  const ArgErr e = validate(m, n, A, lda, sketch_rows, Q, ldq, R, ldr);
  switch (e) {
    case E_OK: break;
    case E_M: return -2;
    case E_N: return -3;
    case E_A: return -4;
    case E_LDA: return -5;
    case E_S: return -6;
    case E_Q: return -9;
    case E_LDQ: return -10;
    case E_R: return -11;
    case E_LDR: return -12;
  }
  if (!work) return -13;
  if (n > kMaxN) return TSQR_ERR_UNSUPPORTED;
  if (work_bytes < make_layout(m, n, sketch_rows).total) return TSQR_ERR_WORKSPACE;
  return run_chain(variant, m, n, A, lda, sketch_rows, seed, extra_pass != 0, Q, ldq, R, ldr, work,
                   d_info, (hipStream_t)stream, 1);
}

int tsqr_sketch_rows(int64_t m, int64_t n, const double* A, int64_t lda, int64_t s,
                     uint64_t seed, double* B, int64_t ldb, void* stream) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (!A) return -3;
  if (lda < m) return -4;
  if (s < 1 || s > kMaxSketchRows) return -5;
  if (!B) return -7;
  if (ldb < s) return -8;
  if (launch_sketch_rows(m, (int)n, A, lda, (int)s, seed, B, ldb, (hipStream_t)stream) !=
      hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

size_t tsqr_cholqr_workspace_bytes(int64_t m, int64_t n) {
  if (n < 1 || n > kMaxN || m < n) return 0;
  return make_chol_layout(m, n).total;
}

int tsqr_cholqr_ws(int algo, int64_t m, int64_t n, const double* A, int64_t lda, double shift,
                   double* Q, int64_t ldq, double* R, int64_t ldr, void* work, size_t work_bytes,
                   int* d_info, void* stream) {
  if (algo != TSQR_ALGO_CHOLQR && algo != TSQR_ALGO_CHOLQR2 && algo != TSQR_ALGO_SCHOLQR3)
    return -1;
  const ArgErr e = validate(m, n, A, lda, n, Q, ldq, R, ldr);
  switch (e) {
    case E_OK: break;
    case E_M: return -2;
    case E_N: return -3;
    case E_A: return -4;
    case E_LDA: return -5;
    case E_S: return -3;
    case E_Q: return -7;
    case E_LDQ: return -8;
    case E_R: return -9;
    case E_LDR: return -10;
  }
  if (!(shift == shift)) return -6;
  if (!work) return -11;
  if (n > kMaxN) return TSQR_ERR_UNSUPPORTED;
  if (work_bytes < make_chol_layout(m, n).total) return TSQR_ERR_WORKSPACE;
  const int npass = algo;  // 1, 2 or 3 passes
  return run_cholqr(npass, algo == TSQR_ALGO_SCHOLQR3, m, n, A, lda, shift, Q, ldq, R, ldr,
                    work, d_info, (hipStream_t)stream);
}

size_t tsqr_lstsq_workspace_bytes(int64_t m, int64_t n, int64_t sketch_rows) {
  if (n < 1 || n > kMaxN || m < n || sketch_rows < n || sketch_rows > kMaxSketchRows) return 0;
  return make_lsq_layout(m, n, sketch_rows).total;
}

int tsqr_lstsq_ws(int variant, int sketch, int64_t m, int64_t n, const double* A, int64_t lda,
                  const double* b, int64_t sketch_rows, uint64_t seed, double* x, void* work,
                  size_t work_bytes, int* d_info, void* stream) {
  if (variant != TSQR_VARIANT_RQR && variant != TSQR_VARIANT_RLU) return -1;
  if (sketch != TSQR_SKETCH_GAUSSIAN && sketch != TSQR_SKETCH_ROWS) return -2;
  if (n < 1) return -4;
  if (m < 1 || m < n) return -3;
  if (!A) return -5;
  if (lda < m) return -6;
  if (!b) return -7;
  if (sketch_rows < n || sketch_rows > kMaxSketchRows) return -8;
  if (!x) return -10;
  if (!work) return -11;
  if (n > kMaxN) return TSQR_ERR_UNSUPPORTED;
  if (work_bytes < make_lsq_layout(m, n, sketch_rows).total) return TSQR_ERR_WORKSPACE;
  return run_lstsq(variant, sketch, m, n, A, lda, b, sketch_rows, seed, x, work, d_info,
                   (hipStream_t)stream);
}

size_t tsqr_mixed_workspace_bytes(int64_t m, int64_t n, int64_t sketch_rows, int lowp) {
  if (n < 1 || n > kMaxNLowp || m < n || sketch_rows < n || sketch_rows > kMaxSketchRows) return 0;
  if (lowp != TSQR_LOWP_FP32 && lowp != TSQR_LOWP_BF16) return 0;
  return make_mixed_layout(m, n, sketch_rows, lowp).total;
}

int tsqr_rxr_cholqr_mixed_ws(int variant, int lowp, int64_t m, int64_t n, const double* A,
                             int64_t lda, int64_t sketch_rows, uint64_t seed, int fp64_passes,
                             double* Q, int64_t ldq, double* R, int64_t ldr, void* work,
                             size_t work_bytes, int* d_info, int* d_report, void* stream) {
  if (variant != TSQR_VARIANT_RQR && variant != TSQR_VARIANT_RLU) return -1;
  if (lowp != TSQR_LOWP_FP32 && lowp != TSQR_LOWP_BF16) return -2;
  const ArgErr e = validate(m, n, A, lda, sketch_rows, Q, ldq, R, ldr);
  switch (e) {
    case E_OK: break;
    case E_M: return -3;
    case E_N: return -4;
    case E_A: return -5;
    case E_LDA: return -6;
    case E_S: return -7;
    case E_Q: return -10;
    case E_LDQ: return -11;
    case E_R: return -12;
    case E_LDR: return -13;
  }
  if (fp64_passes < 0 || fp64_passes > 3) return -9;
  if (!work) return -14;
  if (n > kMaxNLowp) return TSQR_ERR_UNSUPPORTED;
  if (work_bytes < make_mixed_layout(m, n, sketch_rows, lowp).total) return TSQR_ERR_WORKSPACE;
  return run_chain_mixed(variant, lowp, m, n, A, lda, sketch_rows, seed, fp64_passes, Q, ldq, R,
                         ldr, work, d_info, d_report, (hipStream_t)stream);
}

int tsqr_sketch_lowp(int lowp, int64_t m, int64_t n, const double* A, int64_t lda, int64_t s,
                     uint64_t seed, double* B, int64_t ldb, void* work, size_t work_bytes,
                     void* stream) {
  if (lowp != TSQR_LOWP_FP32 && lowp != TSQR_LOWP_BF16) return -1;
  if (m < 1) return -2;
  if (n < 1 || n > kMaxNLowp) return -3;
  if (!A) return -4;
  if (lda < m) return -5;
  if (s < 1 || s > kMaxSketchRows) return -6;
  if (!B) return -8;
  if (ldb < s) return -9;
  if (!work) return -10;
  const SketchPlan p = plan_sketch(m, (int)n, (int)s);
  if (work_bytes < p.part_doubles * sizeof(double)) return TSQR_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  if (launch_sketch_lowp(lowp, p, m, (int)n, A, lda, seed, (double*)work, st) != hipSuccess ||
      launch_sketch_reduce(p, (int)s, (int)n, (double*)work, 1.0 / sqrt((double)s), B, ldb, st) !=
          hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

size_t tsqr_rinv_lowp_bytes(int64_t n, int lowp) {
  if (n < 1 || n > kMaxNLowp || (lowp != TSQR_LOWP_FP32 && lowp != TSQR_LOWP_BF16)) return 0;
  return rinv_lowp_bytes(lowp, (int)n);
}

int tsqr_apply_rinv_lowp(int lowp, int64_t m, int64_t n, const double* Y, int64_t ldy,
                         const double* Rinv, int64_t ldr, void* X, int64_t ldx, void* work,
                         size_t work_bytes, void* stream) {
  if (lowp != TSQR_LOWP_FP32 && lowp != TSQR_LOWP_BF16) return -1;
  if (m < 1) return -2;
  if (n < 1 || n > kMaxNLowp) return -3;
  if (!Y) return -4;
  if (ldy < m) return -5;
  if (!Rinv) return -6;
  if (ldr < n) return -7;
  if (!X) return -8;
  if (ldx < m) return -9;
  if (!work) return -10;
  if (work_bytes < rinv_lowp_bytes(lowp, (int)n)) return TSQR_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  if (launch_rinv_prep(lowp, (int)n, Rinv, ldr, work, st) != hipSuccess ||
      launch_apply_rinv_lowp(lowp, m, (int)n, Y, ldy, work, X, ldx, st) != hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

int tsqr_gram_lowp(int lowp, int64_t m, int64_t n, const void* X, int64_t ldx, double* W,
                   int64_t ldw, void* work, size_t work_bytes, void* stream) {
  if (lowp != TSQR_LOWP_FP32 && lowp != TSQR_LOWP_BF16) return -1;
  if (m < 1) return -2;
  if (n < 1 || n > kMaxNLowp) return -3;
  if (!X) return -4;
  if (ldx < m) return -5;
  if (!W) return -6;
  if (ldw < n) return -7;
  if (!work) return -8;
  const GramPlan p = plan_gram(m, (int)n);
  if (work_bytes < p.part_doubles * sizeof(double)) return TSQR_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  if (launch_gram_lowp(lowp, p, m, (int)n, X, ldx, (double*)work, st) != hipSuccess ||
      launch_gram_reduce(p, (int)n, (double*)work, W, ldw, st) != hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

size_t tsqr_sketch_workspace_bytes(int64_t m, int64_t n, int64_t s) {
  if (m < 1 || n < 1 || s < 1) return 0;
  return plan_sketch(m, (int)n, (int)s).part_doubles * sizeof(double);
}

int tsqr_sketch(int64_t m, int64_t n, const double* A, int64_t lda, int64_t s, uint64_t seed,
                double* B, int64_t ldb, void* work, size_t work_bytes, void* stream) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (!A) return -3;
  if (lda < m) return -4;
  if (s < 1 || s > kMaxSketchRows) return -5;
  if (!B) return -7;
  if (ldb < s) return -8;
  if (!work) return -9;
  const SketchPlan p = plan_sketch(m, (int)n, (int)s);
  if (work_bytes < p.part_doubles * sizeof(double)) return TSQR_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  if (launch_sketch(p, m, (int)n, A, lda, (int)s, seed, (double*)work, st) != hipSuccess)
    return TSQR_ERR_HIP;
  if (launch_sketch_reduce(p, (int)s, (int)n, (double*)work, 1.0 / sqrt((double)s), B, ldb, st) !=
      hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

size_t tsqr_sketch_factor_workspace_bytes(int64_t s, int64_t n) {
  if (n < 1 || s < n || s > kMaxSketchRows) return 0;
  return sketch_factor_scratch_doubles((int)s, (int)n) * sizeof(double);
}

int tsqr_sketch_factor(int variant, int64_t s, int64_t n, const double* B, int64_t ldb,
                       double* R0, int64_t ldr, int* d_info, void* work, size_t work_bytes,
                       void* stream) {
  if (variant != TSQR_VARIANT_RQR && variant != TSQR_VARIANT_RLU) return -1;
  if (s < n || s > kMaxSketchRows) return -2;
  if (n < 1) return -3;
  if (!B) return -4;
  if (ldb < s) return -5;
  if (!R0) return -6;
  if (ldr < n) return -7;
  if (!work || work_bytes < sketch_factor_scratch_doubles((int)s, (int)n) * sizeof(double))
    return TSQR_ERR_WORKSPACE;
  if (launch_sketch_factor(variant, (int)s, (int)n, B, ldb, R0, ldr, d_info, (double*)work,
                           (hipStream_t)stream) != hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

size_t tsqr_trsm_workspace_bytes(int64_t n) {
  if (n < 1 || n > kMaxN) return 0;
  return trsm_scratch_doubles((int)n) * sizeof(double);
}

int tsqr_trsm(int64_t m, int64_t n, const double* Y, int64_t ldy, const double* T, int64_t ldt,
              double* X, int64_t ldx, void* work, size_t work_bytes, void* stream) {
  if (m < 0) return -1;
  if (n < 1) return -2;
  if (!Y) return -3;
  if (ldy < m || ldy < 1) return -4;
  if (!T) return -5;
  if (ldt < n) return -6;
  if (!X) return -7;
  if (ldx < m || ldx < 1) return -8;
  if (X != Y && overlaps(X, span_bytes(m > 0 ? m : 1, n, ldx), Y, span_bytes(m > 0 ? m : 1, n, ldy)))
    return -7;
  if (X == Y && ldx != ldy) return -8;
  if (n > kMaxN) return TSQR_ERR_UNSUPPORTED;
  if (!work) return -9;
  if (work_bytes < trsm_scratch_doubles((int)n) * sizeof(double)) return TSQR_ERR_WORKSPACE;
  if (launch_trsm(m, (int)n, Y, ldy, T, ldt, X, ldx, (double*)work, (hipStream_t)stream) !=
      hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

size_t tsqr_gram_workspace_bytes(int64_t m, int64_t n) {
  if (m < 1 || n < 1) return 0;
  return plan_gram(m, (int)n).part_doubles * sizeof(double);
}

int tsqr_gram(int64_t m, int64_t n, const double* X, int64_t ldx, double* W, int64_t ldw,
              void* work, size_t work_bytes, void* stream) {
  if (m < 1) return -1;
  if (n < 1) return -2;
  if (!X) return -3;
  if (ldx < m) return -4;
  if (!W) return -5;
  if (ldw < n) return -6;
  if (!work) return -7;
  if (n > kMaxN) return TSQR_ERR_UNSUPPORTED;
  const GramPlan p = plan_gram(m, (int)n);
  if (work_bytes < p.part_doubles * sizeof(double)) return TSQR_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  if (launch_gram(p, m, (int)n, X, ldx, (double*)work, st) != hipSuccess) return TSQR_ERR_HIP;
  if (launch_gram_reduce(p, (int)n, (double*)work, W, ldw, st) != hipSuccess) return TSQR_ERR_HIP;
  return TSQR_OK;
}

int tsqr_potrf(int64_t n, const double* W, int64_t ldw, double* R, int64_t ldr, int stage,
               int* d_info, void* work, size_t work_bytes, void* stream) {
  if (n < 1 || n > kMaxSketchRows) return -1;
  if (!W) return -2;
  if (ldw < n) return -3;
  if (!R) return -4;
  if (ldr < n) return -5;
  if (stage < 1 || stage > 9) return -6;
  (void)work;  // the factorization runs in place in R: no scratch
  (void)work_bytes;
  if (launch_potrf((int)n, W, ldw, R, ldr, stage, d_info, nullptr, (hipStream_t)stream) !=
      hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

int tsqr_trmm_upper(int64_t n, const double* A, int64_t lda, const double* B, int64_t ldb,
                    double* C, int64_t ldc, void* stream) {
  if (n < 1) return -1;
  if (!A) return -2;
  if (lda < n) return -3;
  if (!B) return -4;
  if (ldb < n) return -5;
  if (!C) return -6;
  if (ldc < n) return -7;
  if (overlaps(C, span_bytes(n, n, ldc), A, span_bytes(n, n, lda)) ||
      overlaps(C, span_bytes(n, n, ldc), B, span_bytes(n, n, ldb)))
    return -6;
  if (launch_trmm_upper((int)n, A, lda, B, ldb, C, ldc, (hipStream_t)stream) != hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

int tsqr_philox4x32_10(int64_t count, const uint32_t* d_ctr, uint64_t seed, uint32_t* d_out,
                       void* stream) {
  if (count < 0) return -1;
  if (count > 0 && !d_ctr) return -2;
  if (count > 0 && !d_out) return -4;
  if (launch_philox_words(count, d_ctr, seed, d_out, (hipStream_t)stream) != hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

int tsqr_sketch_normals(uint64_t seed, int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                        double* Zout, int64_t ldz, void* stream) {
  if (i0 < 0 || i0 + ni > 0xffffffffLL) return -2;
  if (ni < 0) return -3;
  if (j0 < 0) return -4;
  if (nj < 0) return -5;
  if (ni * nj > 0 && !Zout) return -6;
  if (ldz < ni || ldz < 1) return -7;
  if (launch_sketch_normals(seed, i0, ni, j0, nj, Zout, ldz, (hipStream_t)stream) != hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

size_t tsqr_metrics_workspace_bytes(int64_t m, int64_t n) {
  if (m < 1 || n < 1 || n > 65536) return 0;
  return metrics_workspace_bytes(m, (int)n);
}

int tsqr_metrics(int64_t m, int64_t n, const double* A, int64_t lda, const double* Q,
                 int64_t ldq, const double* R, int64_t ldr, double* d_out, void* work,
                 size_t work_bytes, void* stream) {
  if (m < 1) return -1;
  if (n < 1 || n > 65536) return -2;
  if (A && lda < m) return -4;
  if (!Q) return -5;
  if (ldq < m) return -6;
  if (R && ldr < n) return -8;
  if (!d_out) return -9;
  if (!work || work_bytes < metrics_workspace_bytes(m, (int)n)) return TSQR_ERR_WORKSPACE;
  if (launch_metrics(m, (int)n, A, lda, Q, ldq, R, ldr, d_out, work, (hipStream_t)stream) !=
      hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

int tsqr_probe_stream(int kind, const void* src, void* dst, size_t bytes, int wgs_per_cu,
                      int unroll, int nontemporal, double* d_sink, void* stream) {
  if (kind < 0 || kind > 2) return -1;
  if (kind != 1 && !src) return -2;
  if (kind != 0 && !dst) return -3;
  if (bytes < 16) return -4;
  if (wgs_per_cu < 1 || wgs_per_cu > 64) return -5;
  if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8) return -6;
  if (!d_sink) return -8;
  if (launch_probe_stream(kind, src, dst, bytes, wgs_per_cu, unroll, nontemporal, d_sink,
                          (hipStream_t)stream) != hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

int tsqr_probe_mfma(int kind, int waves_per_simd, int chains, int64_t iters, double* d_sink,
                    double* flops, void* stream) {
  if (kind < 0 || kind > 4) return -1;
  if (waves_per_simd != 1 && waves_per_simd != 2 && waves_per_simd != 4 && waves_per_simd != 8)
    return -2;
  if (chains != 4 && chains != 8 && chains != 16) return -3;
  if (iters < 1) return -4;
  if (!d_sink) return -5;
  if (!flops) return -6;
  if (launch_probe_mfma(kind, waves_per_simd, chains, iters, d_sink, flops,
                        (hipStream_t)stream) != hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

}  // extern "C"
