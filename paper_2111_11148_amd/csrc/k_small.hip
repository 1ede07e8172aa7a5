// Small dense factorizations on the critical path of randomized XR-CholeskyQR:
//   * R0 of the l x n sketch by Householder QR (paper Algorithm rQR-CholeskyQR, step 2)
//     or by partial-pivot LU (Algorithm rLU-CholeskyQR, step 2), sign-normalised;
//   * the n x n Cholesky factor of a Gram matrix (Algorithm CholeskyQR, step 2);
//   * products of upper-triangular factors (R = R2 R1 R0) and breakdown poisoning.
//
// Each factorization runs in one 1024-thread workgroup (16 wavefronts).  Wavefront w owns
// columns w, w+16, w+32, ...; lane l owns rows l, l+64, ...  Column k's owner builds the
// step's vector (Householder vector, LU multipliers or Cholesky row) and publishes it in
// LDS; one barrier per step, after which every wavefront updates its own columns.  The
// register-resident variants keep the matrix in VGPRs; the fallback variants keep it in a
// global scratch copy (each column is only ever touched by its owner wavefront).
#include <math.h>

#include "tsqr_device.hpp"
#include "tsqr_launch.hpp"

namespace tsqr {

constexpr int kSmallWaves = 16;
constexpr int kSmallThreads = kSmallWaves * kWave;

// value at `row` of a register-distributed column (row = lane + 64 r), broadcast
template <int RPL>
__device__ __forceinline__ double col_elem(const double (&x)[RPL], int row) {
  double v = 0.0;
#pragma unroll
  for (int r = 0; r < RPL; ++r)
    if (r == (row >> 6)) v = x[r];
  return __shfl(v, row & 63, kWave);
}

template <int CPW, int RPL>
__device__ __forceinline__ void col_select(const double (&col)[CPW][RPL], int qsel,
                                           double (&x)[RPL]) {
#pragma unroll
  for (int r = 0; r < RPL; ++r) x[r] = 0.0;
#pragma unroll
  for (int qc = 0; qc < CPW; ++qc)
    if (qc == qsel)
#pragma unroll
      for (int r = 0; r < RPL; ++r) x[r] = col[qc][r];
}

// Householder reflector of LAPACK's convention for x = (alpha, x2): beta = -sign(alpha)
// ||x|| (sign(0) = +1), tau = (beta - alpha)/beta, v = (1, x2/(alpha - beta)).
__device__ __forceinline__ void house(double alpha, double xnorm2, double& beta, double& tau,
                                      double& scal) {
  if (xnorm2 == 0.0) {
    beta = alpha;
    tau = 0.0;
    scal = 0.0;
  } else {
    const double nrm = sqrt(alpha * alpha + xnorm2);
    beta = (alpha >= 0.0) ? -nrm : nrm;
    tau = (beta - alpha) / beta;
    scal = 1.0 / (alpha - beta);
  }
}

// ================================================================ Householder QR ====
template <int RPL, int CPW>
__global__ __launch_bounds__(kSmallThreads) void k_geqrf_reg(int s, int n,
                                                             const double* __restrict__ B,
                                                             int64_t ldb, double* __restrict__ R,
                                                             int64_t ldr, int* __restrict__ info) {
  __shared__ double vbuf[2][64 * RPL];
  __shared__ double tau_sh[2];
  __shared__ double betas[16 * CPW];
  const int lane = lane_id(), wave = wave_id();
  double col[CPW][RPL];
#pragma unroll
  for (int qc = 0; qc < CPW; ++qc)
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int c = wave + kSmallWaves * qc, i = lane + 64 * r;
      col[qc][r] = (c < n && i < s) ? B[(int64_t)c * ldb + i] : 0.0;
    }

  for (int k = 0; k < n; ++k) {
    const int buf = k & 1;
    if (wave == k % kSmallWaves) {
      double x[RPL];
      col_select(col, k / kSmallWaves, x);
      double part = 0.0, xk = 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i > k && i < s) part += x[r] * x[r];
        if (i == k) xk = x[r];
      }
      const double xnorm2 = wave_sum(part);
      const double alpha = wave_sum(xk);
      double beta, tau, scal;
      house(alpha, xnorm2, beta, tau, scal);
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        vbuf[buf][i] = (i == k) ? 1.0 : ((i > k && i < s) ? x[r] * scal : 0.0);
      }
      if (lane == 0) {
        tau_sh[buf] = tau;
        betas[k] = beta;
      }
    }
    __syncthreads();
    const double tau = tau_sh[buf];
    if (tau != 0.0) {
      double v[RPL];
#pragma unroll
      for (int r = 0; r < RPL; ++r) v[r] = vbuf[buf][lane + 64 * r];
#pragma unroll
      for (int qc = 0; qc < CPW; ++qc) {
        const int c = wave + kSmallWaves * qc;
        if (c > k && c < n) {
          double p = 0.0;
#pragma unroll
          for (int r = 0; r < RPL; ++r) p += v[r] * col[qc][r];
          const double w = wave_sum(p) * tau;
#pragma unroll
          for (int r = 0; r < RPL; ++r) col[qc][r] -= v[r] * w;
        }
      }
    }
  }
  __syncthreads();
  // sign-normalised R0 = diag(sign beta) R
#pragma unroll
  for (int qc = 0; qc < CPW; ++qc) {
    const int c = wave + kSmallWaves * qc;
    if (c >= n) continue;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      if (i >= n) continue;
      double v = 0.0;
      if (i <= c) {
        const double bi = betas[i];
        const double sg = (bi < 0.0) ? -1.0 : 1.0;
        v = (i == c) ? fabs(bi) : sg * col[qc][r];
        if (i == c && !(bi != 0.0)) v = NAN;
      }
      R[(int64_t)c * ldr + i] = v;
    }
  }
  if (threadIdx.x == 0 && info) {
    int bad = 0;
    for (int k = 0; k < n && !bad; ++k)
      if (!(betas[k] != 0.0)) bad = k + 1;
    if (bad && *info == 0) *info = 1000 + bad;
  }
}

// Global-memory fallback (any s <= kMaxS, n <= s): matrix copied to scratch (ld s).
constexpr int kMaxS = 8192;
__global__ __launch_bounds__(kSmallThreads) void k_geqrf_glb(int s, int n,
                                                             const double* __restrict__ B,
                                                             int64_t ldb, double* __restrict__ R,
                                                             int64_t ldr, int* __restrict__ info,
                                                             double* __restrict__ Wk) {
  extern __shared__ double sm[];
  double* vbuf0 = sm;
  double* vbuf1 = sm + s;
  double* tau_sh = sm + 2 * s;
  double* betas = tau_sh + 2;
  const int lane = lane_id(), wave = wave_id();
  // each wavefront copies its own columns (it is the only one to touch them later)
  for (int c = wave; c < n; c += kSmallWaves)
    for (int i = lane; i < s; i += 64) Wk[(int64_t)c * s + i] = B[(int64_t)c * ldb + i];

  for (int k = 0; k < n; ++k) {
    double* vb = (k & 1) ? vbuf1 : vbuf0;
    if (wave == k % kSmallWaves) {
      const double* x = Wk + (int64_t)k * s;
      double part = 0.0;
      for (int i = k + 1 + lane; i < s; i += 64) part += x[i] * x[i];
      const double xnorm2 = wave_sum(part);
      const double alpha = x[k];
      double beta, tau, scal;
      house(alpha, xnorm2, beta, tau, scal);
      for (int i = lane; i < s; i += 64) vb[i] = (i == k) ? 1.0 : (i > k ? x[i] * scal : 0.0);
      if (lane == 0) {
        tau_sh[k & 1] = tau;
        betas[k] = beta;
      }
    }
    __syncthreads();
    const double tau = tau_sh[k & 1];
    if (tau != 0.0) {
      for (int c = wave; c < n; c += kSmallWaves) {
        if (c <= k) continue;
        double* y = Wk + (int64_t)c * s;
        double p = 0.0;
        for (int i = k + lane; i < s; i += 64) p += vb[i] * y[i];
        const double w = wave_sum(p) * tau;
        for (int i = k + lane; i < s; i += 64) y[i] -= vb[i] * w;
      }
    }
  }
  __syncthreads();
  for (int c = wave; c < n; c += kSmallWaves)
    for (int i = lane; i < n; i += 64) {
      double v = 0.0;
      if (i <= c) {
        const double bi = betas[i];
        const double sg = (bi < 0.0) ? -1.0 : 1.0;
        v = (i == c) ? fabs(bi) : sg * Wk[(int64_t)c * s + i];
        if (i == c && !(bi != 0.0)) v = NAN;
      }
      R[(int64_t)c * ldr + i] = v;
    }
  if (threadIdx.x == 0 && info) {
    int bad = 0;
    for (int k = 0; k < n && !bad; ++k)
      if (!(betas[k] != 0.0)) bad = k + 1;
    if (bad && *info == 0) *info = 1000 + bad;
  }
}

// ========================================================== partial-pivot LU =========
// Pivot: first row index of the largest |b_ik| among rows i >= k (NaN counts as largest).
__device__ __forceinline__ bool piv_better(double a, int ia, double b, int ib) {
  // is (a, ia) preferred over (b, ib)?
  const bool an = isnan(a), bn = isnan(b);
  if (an != bn) return an;
  if (!an && a != b) return a > b;
  return ia < ib;
}

__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ov = __shfl_xor(v, off, kWave);
    const int oi = __shfl_xor(idx, off, kWave);
    if (piv_better(ov, oi, v, idx)) {
      v = ov;
      idx = oi;
    }
  }
}

template <int RPL, int CPW>
__global__ __launch_bounds__(kSmallThreads) void k_getrf_reg(int s, int n,
                                                             const double* __restrict__ B,
                                                             int64_t ldb, double* __restrict__ R,
                                                             int64_t ldr, int* __restrict__ info) {
  __shared__ double lbuf[2][64 * RPL];
  __shared__ int piv_sh[2];
  __shared__ double ukk[16 * CPW];
  const int lane = lane_id(), wave = wave_id();
  double col[CPW][RPL];
#pragma unroll
  for (int qc = 0; qc < CPW; ++qc)
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int c = wave + kSmallWaves * qc, i = lane + 64 * r;
      col[qc][r] = (c < n && i < s) ? B[(int64_t)c * ldb + i] : 0.0;
    }

  for (int k = 0; k < n; ++k) {
    const int buf = k & 1;
    if (wave == k % kSmallWaves) {
      double x[RPL];
      col_select(col, k / kSmallWaves, x);
      double bv = -1.0;
      int bi = 0x7fffffff;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        if (i >= k && i < s) {
          const double a = fabs(x[r]);
          if (piv_better(a, i, bv, bi)) {
            bv = a;
            bi = i;
          }
        }
      }
      wave_argmax(bv, bi);
      const int p = bi;
      const double vk = col_elem(x, k), vp = col_elem(x, p);
      const double pivot = vp;
      // multipliers of the swapped column (row p now holds the old row k)
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        const double xi = (i == p) ? vk : x[r];
        lbuf[buf][i] = (i > k && i < s) ? xi / pivot : 0.0;
      }
      if (lane == 0) {
        piv_sh[buf] = p;
        ukk[k] = pivot;
      }
    }
    __syncthreads();
    const int p = piv_sh[buf];
    double l[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) l[r] = lbuf[buf][lane + 64 * r];
    // swap rows k and p in columns >= k; eliminate below row k in columns > k
#pragma unroll
    for (int qc = 0; qc < CPW; ++qc) {
      const int c = wave + kSmallWaves * qc;
      if (c >= k && c < n) {
        const double vk = col_elem(col[qc], k), vp = col_elem(col[qc], p);
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int i = lane + 64 * r;
          double v = col[qc][r];
          if (i == k) v = vp;
          else if (i == p) v = vk;
          if (c > k && i > k) v -= l[r] * vp;
          col[qc][r] = v;
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int qc = 0; qc < CPW; ++qc) {
    const int c = wave + kSmallWaves * qc;
    if (c >= n) continue;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      if (i >= n) continue;
      double v = 0.0;
      if (i <= c) {
        const double ui = ukk[i];
        const double sg = (ui < 0.0) ? -1.0 : 1.0;
        v = (i == c) ? fabs(ui) : sg * col[qc][r];
        if (i == c && !(ui != 0.0)) v = NAN;
      }
      R[(int64_t)c * ldr + i] = v;
    }
  }
  if (threadIdx.x == 0 && info) {
    int bad = 0;
    for (int k = 0; k < n && !bad; ++k)
      if (!(ukk[k] != 0.0)) bad = k + 1;
    if (bad && *info == 0) *info = 1000 + bad;
  }
}

__global__ __launch_bounds__(kSmallThreads) void k_getrf_glb(int s, int n,
                                                             const double* __restrict__ B,
                                                             int64_t ldb, double* __restrict__ R,
                                                             int64_t ldr, int* __restrict__ info,
                                                             double* __restrict__ Wk) {
  extern __shared__ double sm[];
  double* lb0 = sm;
  double* lb1 = sm + s;
  double* ukk = sm + 2 * s;
  int* piv_sh = reinterpret_cast<int*>(ukk + n);
  const int lane = lane_id(), wave = wave_id();
  for (int c = wave; c < n; c += kSmallWaves)
    for (int i = lane; i < s; i += 64) Wk[(int64_t)c * s + i] = B[(int64_t)c * ldb + i];

  for (int k = 0; k < n; ++k) {
    double* lb = (k & 1) ? lb1 : lb0;
    if (wave == k % kSmallWaves) {
      double* x = Wk + (int64_t)k * s;
      double bv = -1.0;
      int bi = 0x7fffffff;
      for (int i = k + lane; i < s; i += 64) {
        const double a = fabs(x[i]);
        if (piv_better(a, i, bv, bi)) {
          bv = a;
          bi = i;
        }
      }
      wave_argmax(bv, bi);
      const int p = bi;
      const double vk = x[k], vp = x[p];
      if (lane == 0) {
        x[k] = vp;
        x[p] = vk;
      }
      const double pivot = vp;
      for (int i = lane; i < s; i += 64) {
        double xi = x[i];
        if (i == k) xi = vp;
        else if (i == p) xi = vk;
        lb[i] = (i > k) ? xi / pivot : 0.0;
      }
      if (lane == 0) {
        piv_sh[k & 1] = p;
        ukk[k] = pivot;
      }
    }
    __syncthreads();
    const int p = piv_sh[k & 1];
    for (int c = wave; c < n; c += kSmallWaves) {
      if (c <= k) continue;
      double* y = Wk + (int64_t)c * s;
      const double vk = y[k], vp = y[p];
      // every lane has read both values before any lane writes
      __builtin_amdgcn_wave_barrier();
      for (int i = k + lane; i < s; i += 64) {
        double v = y[i];
        if (i == k) v = vp;
        else if (i == p) v = vk;
        if (i > k) v -= lb[i] * vp;
        y[i] = v;
      }
    }
  }
  __syncthreads();
  for (int c = wave; c < n; c += kSmallWaves)
    for (int i = lane; i < n; i += 64) {
      double v = 0.0;
      if (i <= c) {
        const double ui = ukk[i];
        const double sg = (ui < 0.0) ? -1.0 : 1.0;
        v = (i == c) ? fabs(ui) : sg * Wk[(int64_t)c * s + i];
        if (i == c && !(ui != 0.0)) v = NAN;
      }
      R[(int64_t)c * ldr + i] = v;
    }
  if (threadIdx.x == 0 && info) {
    int bad = 0;
    for (int k = 0; k < n && !bad; ++k)
      if (!(ukk[k] != 0.0)) bad = k + 1;
    if (bad && *info == 0) *info = 1000 + bad;
  }
}

// ================================================================== Cholesky =========
// Right-looking Cholesky on the full symmetric matrix (both triangles kept current), so
// that the owner of column k holds row k of R as its column: R(k, i) = W(i, k)/r_kk.
// Reads only the upper triangle of W (the lower one is mirrored on load); `shift` is
// added to the diagonal (shifted CholeskyQR; 0 for the plain factorization).
template <int RPL, int CPW>
__global__ __launch_bounds__(kSmallThreads) void k_potrf_reg(int n, const double* __restrict__ W,
                                                             int64_t ldw, double* __restrict__ R,
                                                             int64_t ldr, int stage,
                                                             int* __restrict__ info,
                                                             double shift) {
  __shared__ double rowk[2][64 * RPL];
  __shared__ int fail_sh;
  const int lane = lane_id(), wave = wave_id();
  double col[CPW][RPL];
#pragma unroll
  for (int qc = 0; qc < CPW; ++qc)
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int c = wave + kSmallWaves * qc, i = lane + 64 * r;
      double v = 0.0;
      if (c < n && i < n) v = (i <= c) ? W[(int64_t)c * ldw + i] : W[(int64_t)i * ldw + c];
      if (c == i) v += shift;
      col[qc][r] = v;
    }
  if (threadIdx.x == 0) fail_sh = -1;
  __syncthreads();

  for (int k = 0; k < n; ++k) {
    const int buf = k & 1;
    if (wave == k % kSmallWaves) {
      double x[RPL];
      col_select(col, k / kSmallWaves, x);
      const double d = col_elem(x, k);
      double rkk;
      if (!(d > 0.0)) {
        rkk = NAN;
        if (lane == 0 && fail_sh < 0) fail_sh = k;
      } else {
        rkk = sqrt(d);
      }
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        const double v = (i > k && i < n) ? x[r] / rkk : (i == k ? rkk : 0.0);
        rowk[buf][i] = v;
        if (i < n) R[(int64_t)i * ldr + k] = v;  // row k of R (zero left of the diagonal)
      }
    }
    __syncthreads();
#pragma unroll
    for (int qc = 0; qc < CPW; ++qc) {
      const int c = wave + kSmallWaves * qc;
      if (c > k && c < n) {
        const double rkc = rowk[buf][c];
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int i = lane + 64 * r;
          if (i > k && i < n) col[qc][r] -= rowk[buf][i] * rkc;
        }
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && info && fail_sh >= 0 && *info == 0) *info = 1000 * stage + fail_sh + 1;
}

__global__ __launch_bounds__(kSmallThreads) void k_potrf_glb(int n, const double* __restrict__ W,
                                                             int64_t ldw, double* __restrict__ R,
                                                             int64_t ldr, int stage,
                                                             int* __restrict__ info,
                                                             double* __restrict__ Wk,
                                                             double shift) {
  extern __shared__ double sm[];
  double* rk0 = sm;
  double* rk1 = sm + n;
  __shared__ int fail_sh;
  const int lane = lane_id(), wave = wave_id();
  for (int c = wave; c < n; c += kSmallWaves)
    for (int i = lane; i < n; i += 64)
      Wk[(int64_t)c * n + i] =
          ((i <= c) ? W[(int64_t)c * ldw + i] : W[(int64_t)i * ldw + c]) + (i == c ? shift : 0.0);
  if (threadIdx.x == 0) fail_sh = -1;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    double* rk = (k & 1) ? rk1 : rk0;
    if (wave == k % kSmallWaves) {
      const double* x = Wk + (int64_t)k * n;
      const double d = x[k];
      double rkk;
      if (!(d > 0.0)) {
        rkk = NAN;
        if (lane == 0 && fail_sh < 0) fail_sh = k;
      } else {
        rkk = sqrt(d);
      }
      for (int i = lane; i < n; i += 64) {
        const double v = (i > k) ? x[i] / rkk : (i == k ? rkk : 0.0);
        rk[i] = v;
        R[(int64_t)i * ldr + k] = v;
      }
    }
    __syncthreads();
    for (int c = wave; c < n; c += kSmallWaves) {
      if (c <= k) continue;
      double* y = Wk + (int64_t)c * n;
      const double rkc = rk[c];
      for (int i = k + 1 + lane; i < n; i += 64) y[i] -= rk[i] * rkc;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && info && fail_sh >= 0 && *info == 0) *info = 1000 * stage + fail_sh + 1;
}

// ============================================================ small products =========
// C = A B for upper-triangular A, B: one 16x16 output tile per workgroup, operands
// staged through LDS in 16-wide chunks of the inner index (only k in [i0, j0+16)).
__global__ __launch_bounds__(256) void k_trmm_upper(int n, const double* __restrict__ A,
                                                    int64_t lda, const double* __restrict__ B,
                                                    int64_t ldb, double* __restrict__ C,
                                                    int64_t ldc) {
  __shared__ double as[16][17], bs[16][17];
  const int i0 = 16 * blockIdx.y, j0 = 16 * blockIdx.x;
  const int ti = threadIdx.x % 16, tj = threadIdx.x / 16;
  const int i = i0 + ti, j = j0 + tj;
  double acc = 0.0;
  if (i0 <= j0 + 15) {
    for (int k0 = i0; k0 < j0 + 16 && k0 < n; k0 += 16) {
      const int ka = k0 + tj, kb = k0 + ti;
      as[ti][tj] = (i < n && ka < n && ka >= i) ? A[(int64_t)ka * lda + i] : 0.0;
      bs[ti][tj] = (kb < n && j < n && kb <= j) ? B[(int64_t)j * ldb + kb] : 0.0;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 16; ++k) acc += as[ti][k] * bs[k][tj];
      __syncthreads();
    }
  }
  if (i < n && j < n) C[(int64_t)j * ldc + i] = (i <= j) ? acc : 0.0;
}

__global__ void k_poison(const int* __restrict__ info, int64_t m, int n, double* Q, int64_t ldq,
                         double* R, int64_t ldr) {
  if (*info == 0) return;
  const int64_t tq = m * n, tr = R ? (int64_t)n * n : 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < tq + tr;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < tq) Q[(e / m) * ldq + (e % m)] = NAN;
    else {
      const int64_t f = e - tq;
      R[(f / n) * ldr + (f % n)] = NAN;
    }
  }
}

__global__ void k_set_int(int* p, int v) { *p = v; }

// I (n x n, ld n)
__global__ void k_identity(int n, double* __restrict__ Y) {
  const int64_t total = (int64_t)n * n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    Y[e] = (e % n == e / n) ? 1.0 : 0.0;
}

// C = *flag ? B : A B for upper n x n A, B (the mixed-precision preconditioner R01 falls
// back to R0 when the Cholesky factor of the low-precision Gram matrix broke down).
__global__ __launch_bounds__(256) void k_trmm_or_copy(const int* __restrict__ flag, int n,
                                                      const double* __restrict__ A, int64_t lda,
                                                      const double* __restrict__ B, int64_t ldb,
                                                      double* __restrict__ C, int64_t ldc) {
  __shared__ double as[16][17], bs[16][17];
  const bool copy = *flag != 0;
  const int i0 = 16 * blockIdx.y, j0 = 16 * blockIdx.x;
  const int ti = threadIdx.x % 16, tj = threadIdx.x / 16;
  const int i = i0 + ti, j = j0 + tj;
  double acc = 0.0;
  if (copy) {
    if (i < n && j < n) acc = (i <= j) ? B[(int64_t)j * ldb + i] : 0.0;
  } else if (i0 <= j0 + 15) {
    for (int k0 = i0; k0 < j0 + 16 && k0 < n; k0 += 16) {
      const int ka = k0 + tj, kb = k0 + ti;
      as[ti][tj] = (i < n && ka < n && ka >= i) ? A[(int64_t)ka * lda + i] : 0.0;
      bs[ti][tj] = (kb < n && j < n && kb <= j) ? B[(int64_t)j * ldb + kb] : 0.0;
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 16; ++k) acc += as[ti][k] * bs[k][tj];
      __syncthreads();
    }
  }
  if (i < n && j < n) C[(int64_t)j * ldc + i] = (i <= j) ? acc : 0.0;
}

// *need = 1 when the preconditioned matrix Q1 with Gram W = Q1^T Q1 is not close enough
// to orthonormal for one CholeskyQR pass (||W - I||_F > thresh), or when `lp_info` or
// `info` report a breakdown.  One workgroup.
__global__ __launch_bounds__(256) void k_pass_decide(int n, const double* __restrict__ W,
                                                     int64_t ldw, const int* __restrict__ lp_info,
                                                     const int* __restrict__ info, double thresh,
                                                     int* __restrict__ need,
                                                     double* __restrict__ dev_out) {
  __shared__ double red[256], red2[256];
  double acc = 0.0, acc2 = 0.0;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e % n, j = e / n;
    const double w = W[(int64_t)j * ldw + i];
    const double d = w - (i == j ? 1.0 : 0.0);
    acc += d * d;
    acc2 += w * w;
  }
  red[threadIdx.x] = acc;
  red2[threadIdx.x] = acc2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x] += red[threadIdx.x + s];
      red2[threadIdx.x] += red2[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double dev = sqrt(red[0]);
    *need = ((lp_info && *lp_info) || (info && *info) || !(dev <= thresh)) ? 1 : 0;
    if (dev_out) {
      dev_out[0] = dev;            // ||W - I||_F
      dev_out[1] = sqrt(red2[0]);  // ||W||_F
    }
  }
}

// ================================================================== launchers ========
static int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

hipError_t launch_sketch_factor(int variant, int s, int n, const double* B, int64_t ldb,
                                double* R, int64_t ldr, int* info, double* scratch,
                                hipStream_t st) {
  const int rpl = pow2_at_least((s + 63) / 64), cpw = pow2_at_least((n + 15) / 16);
  dim3 grid(1), block(kSmallThreads);
#define TSQR_FAC(RPL_, CPW_)                                                                  \
  if (rpl == RPL_ && cpw == CPW_) {                                                           \
    if (variant == 1)                                                                         \
      hipLaunchKernelGGL((k_getrf_reg<RPL_, CPW_>), grid, block, 0, st, s, n, B, ldb, R, ldr, \
                         info);                                                               \
    else                                                                                      \
      hipLaunchKernelGGL((k_geqrf_reg<RPL_, CPW_>), grid, block, 0, st, s, n, B, ldb, R, ldr, \
                         info);                                                               \
    return hipGetLastError();                                                                 \
  }
  TSQR_FAC(1, 1) TSQR_FAC(1, 2) TSQR_FAC(1, 4) TSQR_FAC(1, 8)
  TSQR_FAC(2, 1) TSQR_FAC(2, 2) TSQR_FAC(2, 4) TSQR_FAC(2, 8)
  TSQR_FAC(4, 1) TSQR_FAC(4, 2) TSQR_FAC(4, 4) TSQR_FAC(4, 8)
  TSQR_FAC(8, 1) TSQR_FAC(8, 2) TSQR_FAC(8, 4)
#undef TSQR_FAC
  if (s > kMaxS) return hipErrorInvalidValue;
  if (variant == 1) {
    const size_t sh = (size_t)(2 * s + n) * sizeof(double) + 2 * sizeof(int);
    hipLaunchKernelGGL(k_getrf_glb, grid, block, sh, st, s, n, B, ldb, R, ldr, info, scratch);
  } else {
    const size_t sh = (size_t)(2 * s + 2 + n) * sizeof(double);
    hipLaunchKernelGGL(k_geqrf_glb, grid, block, sh, st, s, n, B, ldb, R, ldr, info, scratch);
  }
  return hipGetLastError();
}

hipError_t launch_potrf(int n, const double* W, int64_t ldw, double* R, int64_t ldr, int stage,
                        int* info, double* scratch, hipStream_t st, double shift) {
  const int rpl = pow2_at_least((n + 63) / 64), cpw = pow2_at_least((n + 15) / 16);
  dim3 grid(1), block(kSmallThreads);
#define TSQR_POTRF(RPL_, CPW_)                                                                 \
  if (rpl == RPL_ && cpw == CPW_) {                                                            \
    hipLaunchKernelGGL((k_potrf_reg<RPL_, CPW_>), grid, block, 0, st, n, W, ldw, R, ldr, stage, \
                       info, shift);                                                           \
    return hipGetLastError();                                                                  \
  }
  TSQR_POTRF(1, 1) TSQR_POTRF(1, 2) TSQR_POTRF(1, 4) TSQR_POTRF(2, 8)
#undef TSQR_POTRF
  if (n > kMaxS) return hipErrorInvalidValue;
  const size_t sh = (size_t)(2 * n) * sizeof(double);
  hipLaunchKernelGGL(k_potrf_glb, grid, block, sh, st, n, W, ldw, R, ldr, stage, info, scratch,
                     shift);
  return hipGetLastError();
}

hipError_t launch_trmm_upper(int n, const double* A, int64_t lda, const double* B, int64_t ldb,
                             double* C, int64_t ldc, hipStream_t st) {
  const int nb = (n + 15) / 16;
  hipLaunchKernelGGL(k_trmm_upper, dim3(nb, nb), dim3(256), 0, st, n, A, lda, B, ldb, C, ldc);
  return hipGetLastError();
}

hipError_t launch_poison(const int* info, int64_t m, int n, double* Q, int64_t ldq, double* R,
                         int64_t ldr, hipStream_t st) {
  hipLaunchKernelGGL(k_poison, dim3(1024), dim3(256), 0, st, info, m, n, Q, ldq, R, ldr);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, st, p, v);
  return hipGetLastError();
}

hipError_t launch_identity(int n, double* Y, hipStream_t st) {
  int blocks = (n * n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_identity, dim3(blocks), dim3(256), 0, st, n, Y);
  return hipGetLastError();
}

hipError_t launch_trmm_or_copy(const int* flag, int n, const double* A, int64_t lda,
                               const double* B, int64_t ldb, double* C, int64_t ldc,
                               hipStream_t st) {
  const int nb = (n + 15) / 16;
  hipLaunchKernelGGL(k_trmm_or_copy, dim3(nb, nb), dim3(256), 0, st, flag, n, A, lda, B, ldb, C,
                     ldc);
  return hipGetLastError();
}

hipError_t launch_pass_decide(int n, const double* W, int64_t ldw, const int* lp_info,
                              const int* info, double thresh, int* need, double* dev_out,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_pass_decide, dim3(1), dim3(256), 0, st, n, W, ldw, lp_info, info, thresh,
                     need, dev_out);
  return hipGetLastError();
}

}  // namespace tsqr
