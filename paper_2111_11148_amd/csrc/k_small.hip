// Small dense factorizations on the critical path of randomized XR-CholeskyQR:
//   * R0 of the l x n sketch by Householder QR (paper Algorithm rQR-CholeskyQR) or by
//     partial-pivot LU (Algorithm rLU-CholeskyQR), sign-normalised;
//   * the n x n Cholesky factor of a Gram matrix (Algorithm CholeskyQR);
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

// value at a uniform `row` of a register-distributed column (row = lane + 64 r), as a
// scalar: every register's lane is read and the scalar selected, so that no register is
// indexed by a run-time value (which would move the column to scratch memory)
template <int RPL>
__device__ __forceinline__ double col_read(const double (&x)[RPL], int row) {
  const int l = row & 63, rr = row >> 6;
  double v = readlane_f64(x[0], l);
#pragma unroll
  for (int r = 1; r < RPL; ++r) {
    const double t = readlane_f64(x[r], l);
    v = (rr == r) ? t : v;
  }
  return v;
}

// x(row) = v for a uniform `row`: one lane of one register replaced (a select in every
// register, for the same reason)
template <int RPL>
__device__ __forceinline__ void col_write(double (&x)[RPL], int row, double v) {
  const bool mine = lane_id() == (row & 63);
  const int rr = row >> 6;
#pragma unroll
  for (int r = 0; r < RPL; ++r) x[r] = (mine && rr == r) ? v : x[r];
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

// 1 + the smallest k < n with a zero or NaN d(k) (neither d > 0 nor d < 0; note that
// NaN != 0 holds, so a test of d != 0 would miss NaN), 0 if there is none;
// the same value in every thread.  Every thread of the workgroup must call it (it has
// barriers); each thread scans a strided share, so no thread walks the whole diagonal.
template <class F>
__device__ __forceinline__ int block_first_bad(int n, F d) {
  __shared__ int best;
  if (threadIdx.x == 0) best = 0x7fffffff;
  __syncthreads();
  int mine = 0x7fffffff;
  for (int k = (int)threadIdx.x; k < n; k += (int)blockDim.x) {
    const double dk = d(k);
    if (!(dk > 0.0 || dk < 0.0)) {
      mine = k;  // strided scan: a thread's first hit is its smallest
      break;
    }
  }
  if (mine != 0x7fffffff) atomicMin(&best, mine);
  __syncthreads();
  return best == 0x7fffffff ? 0 : best + 1;
}

// LDS of the register-resident factorizations of the sketch (QR and LU): two column
// buffers of 64 RPL doubles and one diagonal of 16 CPW.  EXTL bodies take it at ext_lds
// (reg_factor_lds_doubles<RPL, CPW>() doubles) instead of in their own LDS.
template <int RPL, int CPW>
__host__ __device__ constexpr int reg_factor_lds_doubles() {
  return 2 * 64 * RPL + 16 * CPW;
}

// ================================================================ Householder QR ====
// Update of column slots Q0 .. CPW-1 of one wavefront by the step's reflector, with the
// CPW - Q0 dot products summed over the 64 lanes together:
//   * each lane's partial products go to LDS (one padded row per lane, in the
//     wavefront's own region xw of 64 * 9 doubles);
//   * lane l reads back the partials of slot l / G from lanes g, g + G, ... in that order
//     (G = 64 / slots, g = l % G);
//   * the G lanes of a slot add their values by DPP: pairs that differ in lane bit 0, then
//     bit 1, then the mirrored halves of 8 and of 16 lanes, so that each lane ends with
//     the same sum;
//   * slot q's total is read from lane G q (with 32 lanes a slot, the sums of its two rows
//     of 16 are read and added).
// One LDS round trip and a few DPP stages replace a 64-lane reduction per column, and no
// barrier is needed (only this wavefront touches xw, and its LDS operations complete in
// order).  Only columns c > kdone change: a slot with c <= kdone gets w = 0 and is left as
// it is.
template <int RPL, int CPW, int Q0>
__device__ __forceinline__ void qr_slots_update(double (&col)[CPW][RPL], const double (&v)[RPL],
                                                double tau, int kdone, int wave, int lane,
                                                double* xw) {
  constexpr int NQ = CPW - Q0;  // 8, 4 or 2 slots
  constexpr int ST = NQ + 1;    // padded LDS row of one lane
  constexpr int G = 64 / NQ;    // lanes per slot in the transposed sum
  static_assert(NQ == 8 || NQ == 4 || NQ == 2, "transposed sum over 8, 16 or 32 lanes");
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double p = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) p += v[r] * col[Q0 + q][r];
    xw[lane * ST + q] = p;
  }
  const int c = lane / G, g = lane % G;
  double x = 0.0;
#pragma unroll
  for (int i = 0; i < NQ; ++i) x += xw[(g + G * i) * ST + c];
  x += dpp_f64<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp_f64<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp_f64<0x141>(x);  // row_half_mirror: lane i <-> 7 - i within 8
  if constexpr (G >= 16) x += dpp_f64<0x140>(x);  // row_mirror: i <-> 15 - i within 16
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    // 32 lanes per slot: the sums of its two rows of 16 lanes, added in lane order
    double S = readlane_f64(x, G * q);
    if constexpr (G == 32) S = S + readlane_f64(x, G * q + 16);
    const int cq = wave + kSmallWaves * (Q0 + q);
    const double w = (cq > kdone) ? S * tau : 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) col[Q0 + q][r] -= v[r] * w;
  }
}

// XP: the column slots of a wavefront (four or eight) updated together by qr_slots_update
// (the single-problem kernel); otherwise one 64-lane reduction per open column.
template <int RPL, int CPW, bool EXTL = false, bool XP = false>
__device__ __forceinline__ void geqrf_reg_body(int s, int n,
                                                             const double* __restrict__ B,
                                                             int64_t ldb, double* __restrict__ R,
                                                             int64_t ldr, int* __restrict__ info,
                                                             double* ext_lds = nullptr) {
  double* lbase;
  if constexpr (EXTL) {
    lbase = ext_lds;
  } else {
    __shared__ double own[reg_factor_lds_doubles<RPL, CPW>()];
    lbase = own;
  }
  double(*vbuf)[64 * RPL] = reinterpret_cast<double(*)[64 * RPL]>(lbase);
  double* betas = lbase + 2 * 64 * RPL;
  __shared__ double tau_sh[2];
  const int lane = lane_id(), wave = wave_id();
  double* xw = nullptr;
  if constexpr (XP) {
    static_assert(CPW == 8 || CPW == 4, "the transposed update covers four or eight slots");
    __shared__ double xpose[kSmallWaves * 64 * 9];
    xw = xpose + wave * 64 * 9;
  }
  double col[CPW][RPL];
#pragma unroll
  for (int qc = 0; qc < CPW; ++qc)
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int c = wave + kSmallWaves * qc, i = lane + 64 * r;
      col[qc][r] = (c < n && i < s) ? B[(int64_t)c * ldb + i] : 0.0;
    }

  // reflector of column kk by its owner wavefront, published in LDS buffer kk & 1
  auto reflect = [&](int kk) {
    const int buf = kk & 1;
    double x[RPL];
    col_select(col, kk / kSmallWaves, x);
    double part = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      part += (i > kk && i < s) ? x[r] * x[r] : 0.0;
    }
    const double xnorm2 = wave_sum(part);
    const double alpha = col_read(x, kk);
    double beta, tau, scal;
    house(alpha, xnorm2, beta, tau, scal);
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      vbuf[buf][i] = (i == kk) ? 1.0 : ((i > kk && i < s) ? x[r] * scal : 0.0);
    }
    if (lane == 0) {
      tau_sh[buf] = tau;
      betas[kk] = beta;
    }
  };

  for (int k = 0; k < n; ++k) {
    const int buf = k & 1;
    if (wave == k % kSmallWaves) reflect(k);
    __syncthreads();
    const double tau = tau_sh[buf];
    if (tau != 0.0) {
      double v[RPL];
#pragma unroll
      for (int r = 0; r < RPL; ++r) v[r] = vbuf[buf][lane + 64 * r];
      if constexpr (XP) {
        // the first half of the slots holds columns up to 16 * CPW / 2 - 1: all finished
        // from that step on
        if (k < kSmallWaves * (CPW / 2) - 1)
          qr_slots_update<RPL, CPW, 0>(col, v, tau, k, wave, lane, xw);
        else
          qr_slots_update<RPL, CPW, CPW / 2>(col, v, tau, k, wave, lane, xw);
      } else {
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
  if (info) {
    const int bad = block_first_bad(n, [&](int k) { return betas[k]; });
    if (threadIdx.x == 0 && bad && *info == 0) *info = 1000 + bad;
  }
}

template <int RPL, int CPW>
__global__ __launch_bounds__(kSmallThreads) void k_geqrf_reg(int s, int n,
                                                             const double* __restrict__ B,
                                                             int64_t ldb, double* __restrict__ R,
                                                             int64_t ldr, int* __restrict__ info) {
  // the transposed update from two rows per lane (measured: 256 x 128, 229 -> 170 us;
  // 128 x 64, 67 -> 57 us; at one row per lane, 64 x 40, 33 -> 36 us, so not there)
  geqrf_reg_body<RPL, CPW, false, RPL >= 2 && (CPW == 8 || CPW == 4)>(s, n, B, ldb, R, ldr,
                                                                      info);
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
  if (info) {
    const int bad = block_first_bad(n, [&](int k) { return betas[k]; });
    if (threadIdx.x == 0 && bad && *info == 0) *info = 1000 + bad;
  }
}

// ====================================================== blocked Householder QR =====
// For sketches too large for the register-resident kernel: panels of NB columns.  The
// panel kernel (one workgroup) factors rows j0.. of NB columns in LDS with the same
// reflectors as above, and forms the compact-WY factor T of the panel's block reflector
// (H_0 H_1 ... = I - V T V^T; T upper, T_kk = tau_k, T(0:k, k) = -tau_k T(0:k, 0:k)
// V(:, 0:k)^T v_k).  The update kernel applies the block reflector's transpose to the
// trailing columns, C = C - V (T^T (V^T C)), one wavefront per column.  The R entries
// (upper triangle) accumulate in the working copy Wk (ld s); the diagonal is kept in
// `betas`; the finish kernel writes the sign-normalised R0.
// Working space: Wk s*n, V s*NB, T NB*NB, betas n (see qr_blocked_scratch_doubles).
// dst(i, c) = src(i, c) for i < rows, c < cols (src ld lds, dst ld ldd), eight loads in
// flight per thread so the copy is not a chain of memory latencies
__device__ __forceinline__ void copy_to_lds(const double* __restrict__ src, int64_t lds_, int rows,
                                            int cols, double* dst, int ldd) {
  const int total = rows * cols;
  for (int e0 = threadIdx.x; e0 < total; e0 += 8 * (int)blockDim.x) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      const int c = e / rows, i = e - c * rows;
      v[u] = (e < total) ? src[(int64_t)c * lds_ + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * (int)blockDim.x;
      const int c = e / rows, i = e - c * rows;
      if (e < total) dst[c * ldd + i] = v[u];
    }
  }
}

template <int NB>
__host__ __device__ constexpr size_t qr_panel_lds_doubles(int p) {
  return (size_t)NB * (p + 1) + 2 * NB * NB + 2 * NB;
}

template <int NB, int PR>  // PR: rows per lane, s <= 64 PR
__global__ __launch_bounds__(kSmallThreads) void k_qr_panel(int s, int n, int j0,
                                                            double* __restrict__ Wk,
                                                            double* __restrict__ Vb,
                                                            double* __restrict__ Tb,
                                                            double* __restrict__ betas) {
  extern __shared__ double sm[];
  const int p = s - j0;                  // panel rows
  const int w = min(NB, n - j0);         // panel columns
  const int ldp = p + 1;
  double* P = sm;                        // column c at P + c * ldp
  double* G = P + (size_t)NB * ldp;      // G[j * NB + k] = v_j^T v_k (j < k)
  double* T = G + NB * NB;               // T[j * NB + k]
  double* tau = T + NB * NB;
  double* bet = tau + NB;
  const int lane = lane_id(), wave = wave_id();
  copy_to_lds(Wk + (int64_t)j0 * s + j0, s, p, w, P, ldp);
  __syncthreads();
  // Row loops are branch-free so that a lane's eight LDS loads are in flight together: a
  // row past the panel reads and writes the padding entry (row p) of its column, which
  // never enters a sum.
  // reflector of column k from rows k.. of its (updated) column: v = (1, x2 scal)
  auto reflector = [&](int k) {
    double* x = P + k * ldp;
    double part = 0.0;
    for (int r0 = 0; r0 < PR; r0 += 8) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int i = k + 1 + lane + kWave * (r0 + r);
        const double v = x[i < p ? i : p];
        part += (i < p) ? v * v : 0.0;
      }
    }
    const double xnorm2 = wave_sum(part);
    const double alpha = x[k];
    double beta, tk, scal;
    house(alpha, xnorm2, beta, tk, scal);
    for (int r0 = 0; r0 < PR; r0 += 8) {
      double v[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int i = k + 1 + lane + kWave * (r0 + r);
        v[r] = x[i < p ? i : p];
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int i = k + 1 + lane + kWave * (r0 + r);
        x[i < p ? i : p] = v[r] * scal;
      }
    }
    if (lane == 0) {
      x[k] = 1.0;
      tau[k] = tk;
      bet[k] = beta;
    }
  };
  if (wave == 0) reflector(0);
  // step k: apply H_k to columns k+1.. (wave 0 takes column k+1 and then builds the next
  // reflector at once, the other waves share the rest), one barrier per step
  for (int k = 0; k < w; ++k) {
    __syncthreads();
    const double* x = P + k * ldp;
    const double tk = tau[k];
    auto apply = [&](int c) {
      double* y = P + c * ldp;
      double d = 0.0;
      for (int r0 = 0; r0 < PR; r0 += 8) {  // eight rows per lane in flight
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int i = k + lane + kWave * (r0 + r);
          const int ii = i < p ? i : p;
          const double xv = x[ii], yv = y[ii];
          d += (i < p) ? xv * yv : 0.0;
        }
      }
      const double wv = wave_sum(d) * tk;
      for (int r0 = 0; r0 < PR; r0 += 8) {
        double xv[8], yv[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int i = k + lane + kWave * (r0 + r);
          const int ii = i < p ? i : p;
          xv[r] = x[ii];
          yv[r] = y[ii];
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int i = k + lane + kWave * (r0 + r);
          y[i < p ? i : p] = yv[r] - xv[r] * wv;
        }
      }
    };
    if (wave == 0) {
      if (k + 1 < w) {
        apply(k + 1);
        reflector(k + 1);
      }
    } else {
      for (int c = k + 1 + wave; c < w; c += kSmallWaves - 1) apply(c);
    }
  }
  __syncthreads();
  // Gram of the reflector vectors (v_j is zero above row j and 1 at row j)
  for (int t = wave; t < w * w; t += kSmallWaves) {
    const int j = t / w, k = t % w;
    if (j >= k) continue;
    double d = 0.0;
    for (int r0 = 0; r0 < PR; r0 += 8) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int i = k + lane + kWave * (r0 + r);
        const int ii = i < p ? i : p;
        const double a = P[j * ldp + ii], b = P[k * ldp + ii];
        d += (i < p) ? a * b : 0.0;
      }
    }
    d = wave_sum(d);
    if (lane == 0) G[j * NB + k] = d;
  }
  __syncthreads();
  if (wave == 0) {
    // lane j builds row j of T; it only reads entries of that row it wrote itself
    for (int k = 0; k < w; ++k) {
      if (lane < k) {
        double z = 0.0;
#pragma unroll 8
        for (int i = lane; i < k; ++i) z += T[lane * NB + i] * G[i * NB + k];
        T[lane * NB + k] = -tau[k] * z;
      } else if (lane == k) {
        T[k * NB + k] = tau[k];
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NB * NB; e += kSmallThreads) {
    const int j = e / NB, k = e % NB;
    Tb[e] = (j <= k && k < w) ? T[e] : 0.0;
  }
  for (int c = 0; c < w; ++c)
    for (int i = threadIdx.x; i < p; i += kSmallThreads) {
      const double v = P[c * ldp + i];
      Vb[(int64_t)c * s + i] = (i < c) ? 0.0 : v;                 // reflector vectors
      if (i < c) Wk[(int64_t)(j0 + c) * s + j0 + i] = v;          // R entries
    }
  if (threadIdx.x < w) betas[j0 + threadIdx.x] = bet[threadIdx.x];
}

template <int NB, int RPL>
__global__ __launch_bounds__(512) void k_qr_update(int s, int n, int j0, int w, int cpb,
                                                   const double* __restrict__ Vb,
                                                   const double* __restrict__ Tb,
                                                   double* __restrict__ Wk) {
  extern __shared__ double sm[];
  const int p = s - j0;
  double* Vs = sm;                      // column k at Vs + k * p
  double* Ts = Vs + (size_t)NB * p;     // NB x NB
  copy_to_lds(Vb, s, p, w, Vs, p);
  for (int e = threadIdx.x; e < NB * NB; e += blockDim.x) Ts[e] = Tb[e];
  __syncthreads();
  const int lane = lane_id(), wave = wave_id();
  const int c0 = j0 + w + (int)blockIdx.x * cpb;
  const int c1 = min(n, c0 + cpb);
  // The update runs only for a full panel (w == NB; a narrower panel is the last one).
  // Branch-free row loops (a lane's loads are all in flight together): a row past the
  // panel reads row 0, a valid address, and enters no sum; only its store is skipped.
  // One column per wavefront (cpb is the number of wavefronts), its RPL rows per lane in
  // registers; rolled loops over the panel's reflectors keep one row of V per lane in
  // flight.  Row loops are branch-free: a row past the panel reads row 0, a valid
  // address, and enters no sum; only its store is skipped.
  __shared__ double ds_[8][NB];  // d = V^T y, then e = T^T d, per wavefront
  const int c = c0 + wave;
  if (c >= c1) return;
  double* y = Wk + (int64_t)c * s + j0;
  double yv[RPL];
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = lane + kWave * r;
    const double v = y[i < p ? i : 0];
    yv[r] = (i < p) ? v : 0.0;
  }
  double* dw = ds_[wave];
#pragma unroll 1
  for (int k = 0; k < NB; ++k) {
    const lds_f64* vk = (const lds_f64*)Vs + k * p;
    double part = 0.0;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + kWave * r;
      part += (i < p) ? vk[i < p ? i : 0] * yv[r] : 0.0;
    }
    part = wave_sum(part);
    if (lane == 0) dw[k] = part;
  }
  __builtin_amdgcn_wave_barrier();
  // e = T^T d (T upper: e_k = sum_{j <= k} T_jk d_j), entry k computed by lane k
  double el = 0.0;
  if (lane < NB)
    for (int j = 0; j <= lane; ++j) el += Ts[j * NB + lane] * dw[j];
  __builtin_amdgcn_wave_barrier();
  if (lane < NB) dw[lane] = el;
  __builtin_amdgcn_wave_barrier();
#pragma unroll 1
  for (int k = 0; k < NB; ++k) {
    const lds_f64* vk = (const lds_f64*)Vs + k * p;
    const double ek = dw[k];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + kWave * r;
      yv[r] -= vk[i < p ? i : 0] * ek;
    }
  }
#pragma unroll
  for (int r = 0; r < RPL; ++r) {
    const int i = lane + kWave * r;
    if (i < p) y[i] = yv[r];
  }
}

// R0 = diag(sign(beta)) R: R(i, c) = sign(beta_i) Wk(i, c) (i < c), |beta_c| on the
// diagonal (NaN when beta_c is zero or NaN), zero below; info = 1000 + first bad column.
__global__ __launch_bounds__(256) void k_qr_finish(int s, int n, const double* __restrict__ Wk,
                                                   const double* __restrict__ betas,
                                                   double* __restrict__ R, int64_t ldr,
                                                   int* __restrict__ info) {
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = 0.0;
    if (i < c) {
      v = (betas[i] < 0.0 ? -1.0 : 1.0) * Wk[(int64_t)c * s + i];
    } else if (i == c) {
      const double b = betas[c];
      v = (b != 0.0) ? fabs(b) : NAN;
    }
    R[(int64_t)c * ldr + i] = v;
  }
  if (c == 0 && info) {
    const int bad = block_first_bad(n, [&](int k) { return betas[k]; });
    if (threadIdx.x == 0 && bad && *info == 0) *info = 1000 + bad;
  }
}

__global__ __launch_bounds__(256) void k_copy_cols(int s, int n, const double* __restrict__ B,
                                                   int64_t ldb, double* __restrict__ Wk) {
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < s; i += blockDim.x) Wk[(int64_t)c * s + i] = B[(int64_t)c * ldb + i];
}

// ========================================================== partial-pivot LU =========
// Pivot: first row index of the largest |b_ik| among rows i >= k (NaN counts as largest).
__device__ __forceinline__ bool piv_better(double a, int ia, double b, int ib) {
  // is (a, ia) preferred over (b, ib)?  (bitwise operators, no short-circuit: compares and
  // selects rather than branches inside the reductions)
  const bool an = isnan(a), bn = isnan(b), first = ia < ib, gt = a > b, eq = a == b;
  return (an & !bn) | (an & bn & first) | (!an & !bn & (gt | (eq & first)));
}

// Maximum of a double over the 64 lanes, the same in every lane: DPP within rows of 16
// lanes (swap pairs, swap halves of quads, rotate by 4 and by 8), then the four row maxima.
// No lane may hold a NaN; all lanes must be active.
__device__ __forceinline__ double wave_max_f64(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));   // quad_perm [1,0,3,2]
  v = fmax(v, dpp_f64<0x4E>(v));   // quad_perm [2,3,0,1]
  v = fmax(v, dpp_f64<0x124>(v));  // row_ror:4
  v = fmax(v, dpp_f64<0x128>(v));  // row_ror:8
  return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)),
              fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// Minimum of an int over the 64 lanes (same pattern), the same in every lane.
template <int CTRL>
__device__ __forceinline__ int dpp_min_i32(int x) {
  return min(x, __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ int wave_min_i32(int x) {
  x = dpp_min_i32<0xB1>(x);
  x = dpp_min_i32<0x4E>(x);
  x = dpp_min_i32<0x124>(x);
  x = dpp_min_i32<0x128>(x);
  return min(min(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16)),
             min(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48)));
}

// The preferred (value, index) pair of the wavefront, in every lane.  piv_better is a total
// order on pairs with distinct indices, so the winner is unique and any way of finding it
// gives the same pair: if some lane holds a NaN, the smallest index among those lanes;
// otherwise the largest value, and the smallest index among the lanes that hold it (a
// maximum and a minimum by DPP, no pairwise comparisons).  The value is read from the
// winning lane.  All lanes must be active.
__device__ __forceinline__ void wave_argmax(double& v, int& idx) {
  const bool nan = isnan(v);
  int cand;
  if (__ballot(nan) != 0ull) {  // uniform
    cand = nan ? idx : 0x7fffffff;
  } else {
    const double m = wave_max_f64(v);
    cand = (v == m) ? idx : 0x7fffffff;
  }
  const int best = wave_min_i32(cand);
  const int src = __builtin_ctzll(__ballot(cand == best));  // some lane holds best
  v = readlane_f64(v, src);
  idx = best;
}

template <int RPL, int CPW, bool EXTL = false>
__device__ __forceinline__ void getrf_reg_body(int s, int n,
                                                             const double* __restrict__ B,
                                                             int64_t ldb, double* __restrict__ R,
                                                             int64_t ldr, int* __restrict__ info,
                                                             double* ext_lds = nullptr) {
  double* lbase;
  if constexpr (EXTL) {
    lbase = ext_lds;
  } else {
    __shared__ double own[reg_factor_lds_doubles<RPL, CPW>()];
    lbase = own;
  }
  double(*lbuf)[64 * RPL] = reinterpret_cast<double(*)[64 * RPL]>(lbase);
  double* ukk = lbase + 2 * 64 * RPL;
  __shared__ int piv_sh[2];
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
      const double vk = col_read(x, k), vp = col_read(x, p);
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
    // swap rows k and p in columns >= k (two lane writes); eliminate below row k in
    // columns > k (the multipliers are zero in rows <= k)
#pragma unroll
    for (int qc = 0; qc < CPW; ++qc) {
      const int c = wave + kSmallWaves * qc;
      if (c >= k && c < n) {
        const double vk = col_read(col[qc], k), vp = col_read(col[qc], p);
        col_write(col[qc], p, vk);
        col_write(col[qc], k, vp);
        if (c > k)
#pragma unroll
          for (int r = 0; r < RPL; ++r) col[qc][r] -= l[r] * vp;
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
  if (info) {
    const int bad = block_first_bad(n, [&](int k) { return ukk[k]; });
    if (threadIdx.x == 0 && bad && *info == 0) *info = 1000 + bad;
  }
}

template <int RPL, int CPW>
__global__ __launch_bounds__(kSmallThreads) void k_getrf_reg(int s, int n,
                                                             const double* __restrict__ B,
                                                             int64_t ldb, double* __restrict__ R,
                                                             int64_t ldr, int* __restrict__ info) {
  getrf_reg_body<RPL, CPW>(s, n, B, ldb, R, ldr, info);
}

// Partial-pivot LU with implicit row interchanges, for s <= 256 rows and four or eight
// column slots per wavefront (layout as in getrf_reg_body).  Rows are never moved: pos (in
// registers, the same in every wavefront) gives the logical position of each physical row
// and perm (LDS) its inverse.  Step k:
//   * the owner of column k takes the pivot among the rows at positions >= k (largest
//     |a|, first position on ties, exactly as with explicit swaps), exchanges positions k
//     and p, and publishes the multipliers of the rows now past position k by physical
//     row, with the pivot's physical row and the exchanged rows;
//   * after the barrier every wavefront updates its positions and its columns c > k by
//     a -= l u, where u is the pivot row's entry of the column: the one lane holding the
//     pivot row writes all its registers to the wavefront's LDS region and every lane
//     reads the register it needs (no lane selects, no barrier: one wavefront's LDS
//     operations complete in order).
// Each entry sees the same operations in the same order as with explicit swaps, so the
// factor is the same; the pivot row of step k keeps its values from then on and is row k
// of U, which the output writes at its logical position.
template <int RPL, int CPW>
__global__ __launch_bounds__(kSmallThreads) void k_getrf_ip(int s, int n,
                                                            const double* __restrict__ B,
                                                            int64_t ldb, double* __restrict__ R,
                                                            int64_t ldr, int* __restrict__ info) {
  __shared__ double lbuf[2][64 * RPL];             // multipliers by physical row
  __shared__ double ukk[kSmallWaves * CPW];        // pivots by step
  __shared__ int perm[64 * RPL];                   // logical position -> physical row
  __shared__ int piv_sh[2][3];                     // pivot row, row at position k, position p
  __shared__ double rowb[kSmallWaves][CPW * RPL];  // the pivot lane's registers, per wavefront
  const int lane = lane_id(), wave = wave_id();
  double col[CPW][RPL];
  int pos[RPL];
#pragma unroll
  for (int qc = 0; qc < CPW; ++qc)
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int c = wave + kSmallWaves * qc, i = lane + 64 * r;
      col[qc][r] = (c < n && i < s) ? B[(int64_t)c * ldb + i] : 0.0;
    }
#pragma unroll
  for (int r = 0; r < RPL; ++r) pos[r] = lane + 64 * r;
  for (int i = threadIdx.x; i < 64 * RPL; i += kSmallThreads) perm[i] = i;
  __syncthreads();

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
        if (pos[r] >= k && i < s) {
          const double a = fabs(x[r]);
          if (piv_better(a, pos[r], bv, bi)) {
            bv = a;
            bi = pos[r];
          }
        }
      }
      wave_argmax(bv, bi);
      const int pl = bi;                        // position of the pivot
      const int pp = perm[pl], pk = perm[k];    // physical rows at positions p and k
      const double pivot = col_read(x, pp);
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int i = lane + 64 * r;
        const int np = (i == pp) ? k : ((i == pk) ? pl : pos[r]);
        lbuf[buf][i] = (np > k && i < s) ? x[r] / pivot : 0.0;
      }
      if (lane == 0) {
        piv_sh[buf][0] = pp;
        piv_sh[buf][1] = pk;
        piv_sh[buf][2] = pl;
        ukk[k] = pivot;
        perm[pl] = pk;
        perm[k] = pp;
      }
    }
    __syncthreads();
    const int pp = piv_sh[buf][0], pk = piv_sh[buf][1], pl = piv_sh[buf][2];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = lane + 64 * r;
      pos[r] = (i == pp) ? k : ((i == pk) ? pl : pos[r]);
    }
    double l[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) l[r] = lbuf[buf][lane + 64 * r];
    double* rw = rowb[wave];
    if (lane == (pp & 63)) {
#pragma unroll
      for (int qc = 0; qc < CPW; ++qc)
#pragma unroll
        for (int r = 0; r < RPL; ++r) rw[qc * RPL + r] = col[qc][r];
    }
    const int rp = pp >> 6;
#pragma unroll
    for (int qc = 0; qc < CPW; ++qc) {
      const int c = wave + kSmallWaves * qc;
      const double u = (c > k) ? rw[qc * RPL + rp] : 0.0;
#pragma unroll
      for (int r = 0; r < RPL; ++r) col[qc][r] -= l[r] * u;
    }
  }
  __syncthreads();
  // sign-normalised R0 = diag(sign u_kk) U: the entries of physical row i go to its
  // logical position (rows of one column stay inside that column's n doubles)
#pragma unroll
  for (int qc = 0; qc < CPW; ++qc) {
    const int c = wave + kSmallWaves * qc;
    if (c >= n) continue;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int i = pos[r];
      if (i >= n || lane + 64 * r >= s) continue;
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
  if (info) {
    const int bad = block_first_bad(n, [&](int k) { return ukk[k]; });
    if (threadIdx.x == 0 && bad && *info == 0) *info = 1000 + bad;
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
  if (info) {
    const int bad = block_first_bad(n, [&](int k) { return ukk[k]; });
    if (threadIdx.x == 0 && bad && *info == 0) *info = 1000 + bad;
  }
}

// ================================================================== Cholesky =========
// Right-looking Cholesky on the full symmetric matrix (both triangles kept current), so
// that the owner of column k holds row k of R as its column: R(k, i) = W(i, k)/r_kk.
// Reads only the upper triangle of W (the lower one is mirrored on load); `shift` is
// added to the diagonal (shifted CholeskyQR; 0 for the plain factorization).
template <int RPL, int CPW>
__device__ __forceinline__ void potrf_reg_body(int n, const double* __restrict__ W,
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

// Blocked Cholesky of n <= kCholLdsMax columns in one workgroup, the whole upper triangle
// resident in LDS (n (n + 1) doubles), 16-row panels:
//  (a) the block row [R11 R12] = R11^{-T} [W11 W12] by right-looking elimination in
//      registers: in each of the wavefronts taking part, lanes 0..15 hold the columns of the
//      diagonal block (the same in every such wavefront) and lanes 16..63 hold 48 columns
//      of the panel row; row k of the factor reaches every lane by lane reads from lanes
//      0..15, so the block needs no LDS round trip or barrier (the panel columns undergo
//      the operations of forward substitution, in the same order);
//  (b) the trailing update W22 -= R12^T R12 on FP64 MFMA, one wavefront per upper 16 x 16
//      tile, operands and accumulators read from and written back to LDS.
// Two barriers per panel; W is read once at the start and R written once at the end, so
// R may be W itself.  A pivot that is not positive (or NaN) becomes a NaN diagonal entry,
// which then fills the rest of the factor; info names the first such column.
constexpr int kCholLdsMax = 128;

__host__ __device__ constexpr size_t chol_lds_bytes(int n) {
  return (size_t)n * (size_t)(n + 1) * sizeof(double);
}

__global__ __launch_bounds__(kSmallThreads) void k_potrf_lds(int n, const double* __restrict__ W,
                                                             int64_t ldw, double* R, int64_t ldr,
                                                             int stage, int* __restrict__ info,
                                                             double shift,
                                                             const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  extern __shared__ double A[];     // column c at A + c * lda, rows 0..n-1
  __shared__ int fail_sh;
  const int lda = n + 1;
  const int lane = lane_id(), wave = wave_id();
  const int q = lane >> 4, c16 = lane & 15;
  for (int e = threadIdx.x; e < n * n; e += kSmallThreads) {
    const int c = e / n, i = e % n;
    A[c * lda + i] = (i <= c) ? W[(int64_t)c * ldw + i] + (i == c ? shift : 0.0) : 0.0;
  }
  if (threadIdx.x == 0) fail_sh = -1;
  __syncthreads();

  for (int j0 = 0; j0 < n; j0 += 16) {
    const int b = min(16, n - j0), t = n - j0 - b;
    // (a) the block row: wavefront w takes panel columns 48 w .. 48 w + 47
    if (wave == 0 || 48 * wave < t) {
      const bool diag = lane < 16;
      const int c = diag ? j0 + lane : j0 + 16 + 48 * wave + (lane - 16);
      const bool cok = diag ? lane < b : c < n;
      const int kmax = diag ? lane : 15;  // rows of this lane's column inside the block row
      double col[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) col[i] = (cok && i <= kmax) ? A[c * lda + j0 + i] : 0.0;
      // Every lane runs every step unmasked: entries below a diagonal lane's own row (and
      // the columns of lanes past the matrix) take values that are never read or stored.
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (k < b) {
          const double dkk = readlane_f64(col[k], k);
          const bool ok = dkk > 0.0;
          const double rkk = ok ? sqrt(dkk) : NAN;
          if (!ok && lane == 0 && wave == 0 && fail_sh < 0) fail_sh = j0 + k;
          const double rkc = col[k] / rkk;  // R(j0 + k, c)
          col[k] = (diag && lane == k) ? rkk : rkc;
#pragma unroll
          for (int i = k + 1; i < 16; ++i)
            col[i] -= readlane_f64(rkc, i) * rkc;  // R(j0 + k, j0 + i) from lane i
        }
      }
      if (cok && (!diag || wave == 0))
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (i <= kmax) A[c * lda + j0 + i] = col[i];
    }
    __syncthreads();
    if (t == 0) break;
    // (b) W22 -= R12^T R12 on the upper tiles (ta, tb) of the trailing block
    const int o = j0 + 16, tt = (t + 15) / 16, nt = tt * (tt + 1) / 2;
    for (int u = wave; u < nt; u += kSmallWaves) {
      int tb = 0;
      while ((tb + 1) * (tb + 2) / 2 <= u) ++tb;
      const int ta = u - tb * (tb + 1) / 2;
      const int ca = o + 16 * ta + c16, cb = o + 16 * tb + c16;
      v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double av = ca < n ? A[ca * lda + j0 + 4 * kk + q] : 0.0;
        const double bv = cb < n ? A[cb * lda + j0 + 4 * kk + q] : 0.0;
        acc = mfma_f64(av, bv, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = o + 16 * ta + 4 * r + q;
        if (cb < n && row <= cb) A[cb * lda + row] -= acc[r];
      }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < n * n; e += kSmallThreads) {
    const int c = e / n, i = e % n;
    R[(int64_t)c * ldr + i] = (i <= c) ? A[c * lda + i] : 0.0;
  }
  if (threadIdx.x == 0 && info && fail_sh >= 0 && *info == 0) *info = 1000 * stage + fail_sh + 1;
}

// ------------------------------------------------------------------------------------
// Blocked Cholesky (n > 64), in place in R: k_chol_init copies the upper triangle of W
// (plus `shift` on the diagonal) to R with zeros below; then for each panel of NB columns
//  (a) one wavefront factors the NB x NB diagonal block: lane c keeps column c in
//      registers, and row k of the factor is published in LDS (one wavefront: no barrier);
//  (b) the panel row R12 = R11^{-T} W12 by forward substitution, one thread per column
//      ((a) and (b) are one workgroup, k_chol_panel);
//  (c) the trailing update W22 -= R12^T R12 on FP64 MFMA over the trailing upper 16 x 16
//      tiles, one wavefront per tile (k_chol_trail).
// The panels are ordered on the stream.  A pivot that is not positive (or NaN) becomes a
// NaN diagonal entry, which then fills the rest of the factor.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_chol_init(int n, const double* __restrict__ W,
                                                   int64_t ldw, double* __restrict__ R,
                                                   int64_t ldr, double shift,
                                                   const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    R[(int64_t)c * ldr + i] = (i <= c) ? W[(int64_t)c * ldw + i] + (i == c ? shift : 0.0) : 0.0;
}

constexpr int kCholPanelThreads = 256;

template <int NB>
__global__ __launch_bounds__(kCholPanelThreads) void k_chol_panel(int n, double* R, int64_t ldr,
                                                              int j0, int stage,
                                                              int* __restrict__ info,
                                                              const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  constexpr int LDD = NB + 1;
  __shared__ double D[NB * LDD];  // D[k * LDD + c] = R11(k, c)
  __shared__ int fail_sh;
  const int lane = lane_id(), wave = wave_id();
  const int b = min(NB, n - j0), t = n - j0 - b;
  if (threadIdx.x == 0) fail_sh = -1;
  __syncthreads();
  if (wave == 0) {
    const int c = lane;
    const bool cok = c < b;
    double col[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) col[i] = (cok && i <= c) ? R[(int64_t)(j0 + c) * ldr + j0 + i] : 0.0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      if (k < b) {
        const double dkk = readlane_f64(col[k], k);
        const bool ok = dkk > 0.0;
        const double rkk = ok ? sqrt(dkk) : NAN;
        if (!ok && lane == 0 && fail_sh < 0) fail_sh = j0 + k;
        double rkc = 0.0;
        if (c == k) rkc = rkk;
        else if (c > k && cok) rkc = col[k] / rkk;
        col[k] = rkc;
        if (c < NB) D[k * LDD + c] = rkc;
        __builtin_amdgcn_wave_barrier();  // row k is read below by every lane
#pragma unroll
        for (int i = k + 1; i < NB; ++i)
          if (i <= c && cok) col[i] -= D[k * LDD + i] * rkc;
      }
    }
#pragma unroll
    for (int i = 0; i < NB; ++i)
      if (cok && i <= c) R[(int64_t)(j0 + c) * ldr + j0 + i] = col[i];
  }
  __syncthreads();
  for (int tc = threadIdx.x; tc < t; tc += kCholPanelThreads) {
    const int cg = j0 + b + tc;  // b == NB whenever t > 0
    // opaque per-column base: R11 would otherwise be hoisted out of the loop into registers
    const lds_f64* Dp = (const lds_f64*)D;
    asm volatile("" : "+v"(Dp));
    double x[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) x[i] = R[(int64_t)cg * ldr + j0 + i];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double acc = x[i];
#pragma unroll
      for (int k = 0; k < i; ++k) acc -= Dp[k * LDD + i] * x[k];
      x[i] = acc / Dp[i * LDD + i];
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) R[(int64_t)cg * ldr + j0 + i] = x[i];
  }
  if (threadIdx.x == 0 && info && fail_sh >= 0 && *info == 0) *info = 1000 * stage + fail_sh + 1;
}

// W22 -= R12^T R12 on the upper 16 x 16 tiles of the trailing matrix: wavefront w of
// workgroup (x, y) updates tile (ta, tb) = (4y + w, x) when ta <= tb.  Operands: lane
// (q, c16) feeds R12(4kk + q, 16ta + c16) and R12(4kk + q, 16tb + c16); accumulator
// register r is tile entry (4r + q, c16).
template <int NB>
__global__ __launch_bounds__(256) void k_chol_trail(int n, double* R, int64_t ldr, int j0,
                                                    const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  const int lane = lane_id(), wave = wave_id();
  const int q = lane >> 4, c16 = lane & 15;
  const int ta = 4 * blockIdx.y + wave, tb = blockIdx.x;
  const int o = j0 + NB, t = n - o;
  if (ta > tb || 16 * ta >= t) return;
  const int ca = 16 * ta + c16, cb = 16 * tb + c16;
  const double* pa = R + (int64_t)(o + (ca < t ? ca : 0)) * ldr + j0 + q;
  const double* pb = R + (int64_t)(o + (cb < t ? cb : 0)) * ldr + j0 + q;
  double av[NB / 4], bv[NB / 4], old[4];
#pragma unroll
  for (int kk = 0; kk < NB / 4; ++kk) {
    av[kk] = ca < t ? pa[4 * kk] : 0.0;
    bv[kk] = cb < t ? pb[4 * kk] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * ta + 4 * r + q;
    old[r] = (row < t && cb < t && row <= cb) ? R[(int64_t)(o + cb) * ldr + o + row] : 0.0;
  }
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < NB / 4; ++kk) acc = mfma_f64(av[kk], bv[kk], acc);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 16 * ta + 4 * r + q;
    if (row < t && cb < t && row <= cb) R[(int64_t)(o + cb) * ldr + o + row] = old[r] - acc[r];
  }
}

template <int NB>
static hipError_t potrf_multi_t(int n, const double* W, int64_t ldw, double* R, int64_t ldr,
                                int stage, int* info, hipStream_t st, double shift,
                                const int* gate) {
  static_assert(NB <= kWave && NB % 4 == 0, "one wavefront factors the diagonal block");
  hipLaunchKernelGGL(k_chol_init, dim3(n), dim3(256), 0, st, n, W, ldw, R, ldr, shift, gate);
  hipError_t e = hipGetLastError();
  for (int j0 = 0; j0 < n && e == hipSuccess; j0 += NB) {
    hipLaunchKernelGGL(k_chol_panel<NB>, dim3(1), dim3(kCholPanelThreads), 0, st, n, R, ldr, j0,
                       stage, info, gate);
    e = hipGetLastError();
    const int t = n - j0 - NB;
    if (t > 0 && e == hipSuccess) {
      const int tt = (t + 15) / 16;
      hipLaunchKernelGGL(k_chol_trail<NB>, dim3(tt, (tt + 3) / 4), dim3(256), 0, st, n, R, ldr,
                         j0, gate);
      e = hipGetLastError();
    }
  }
  return e;
}

// ============================================================ small products =========
// C = A B for upper-triangular A, B: one 16x16 output tile per workgroup.  The operands of
// the inner indices k in [i0, j0+16) (at most 128 of them) are loaded together, eight
// 16-wide chunks per thread in flight, and staged in LDS behind one barrier; each entry then
// sums over k in increasing order (the entries outside the triangles are zeros).
constexpr int kTrmmMaxK = 128;
__device__ __forceinline__ void trmm_upper_body(int n, const double* __restrict__ A,
                                                    int64_t lda, const double* __restrict__ B,
                                                    int64_t ldb, double* __restrict__ C,
                                                    int64_t ldc, int bx, int by) {
  __shared__ double as[16][kTrmmMaxK + 1], bs[kTrmmMaxK][17];
  const int i0 = 16 * by, j0 = 16 * bx;
  const int ti = threadIdx.x % 16, tj = threadIdx.x / 16;
  const int i = i0 + ti, j = j0 + tj;
  double acc = 0.0;
  if (i0 <= j0 + 15) {
    const int kend = min(j0 + 16, n);
    for (int kc = i0; kc < kend; kc += kTrmmMaxK) {  // one round for n <= 128
      double va[kTrmmMaxK / 16], vb[kTrmmMaxK / 16];
#pragma unroll
      for (int u = 0; u < kTrmmMaxK / 16; ++u) {
        const int ka = kc + 16 * u + tj, kb = kc + 16 * u + ti;
        va[u] = (i < n && ka < kend && ka >= i) ? A[(int64_t)ka * lda + i] : 0.0;
        vb[u] = (kb < kend && j < n && kb <= j) ? B[(int64_t)j * ldb + kb] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kTrmmMaxK / 16; ++u) {
        as[ti][16 * u + tj] = va[u];
        bs[16 * u + ti][tj] = vb[u];
      }
      __syncthreads();
      const int nk = min(kTrmmMaxK, ((kend - kc + 15) / 16) * 16);
      for (int k = 0; k < nk; ++k) acc += as[ti][k] * bs[k][tj];
      __syncthreads();
    }
  }
  if (i < n && j < n) C[(int64_t)j * ldc + i] = (i <= j) ? acc : 0.0;
}

__global__ __launch_bounds__(256) void k_trmm_upper(int n, const double* __restrict__ A,
                                                    int64_t lda, const double* __restrict__ B,
                                                    int64_t ldb, double* __restrict__ C,
                                                    int64_t ldc,
                                                    const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  trmm_upper_body(n, A, lda, B, ldb, C, ldc, (int)blockIdx.x, (int)blockIdx.y);
}

__device__ __forceinline__ void poison_body(const int* __restrict__ info, int64_t m, int n, double* Q, int64_t ldq,
                         double* R, int64_t ldr, int bx, int nbx) {
  if (*info == 0) return;
  const int64_t tq = m * n, tr = R ? (int64_t)n * n : 0;
  for (int64_t e = (int64_t)bx * blockDim.x + threadIdx.x; e < tq + tr;
       e += (int64_t)nbx * blockDim.x) {
    if (e < tq) Q[(e / m) * ldq + (e % m)] = NAN;
    else {
      const int64_t f = e - tq;
      R[(f / n) * ldr + (f % n)] = NAN;
    }
  }
}

__global__ void k_poison(const int* __restrict__ info, int64_t m, int n, double* Q, int64_t ldq,
                         double* R, int64_t ldr) {
  poison_body(info, m, n, Q, ldq, R, ldr, (int)blockIdx.x, (int)gridDim.x);
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
__global__ __launch_bounds__(1024) void k_pass_decide(int n, const double* __restrict__ W,
                                                     int64_t ldw, const int* __restrict__ lp_info,
                                                     const int* __restrict__ info, double thresh,
                                                     int* __restrict__ need,
                                                     double* __restrict__ dev_out,
                                                     const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  __shared__ double red[1024], red2[1024];
  double acc = 0.0, acc2 = 0.0;
  // a column per 64-lane group (rows coalesced, no index division)
  const int g = threadIdx.x / 64, ng = blockDim.x / 64;
  for (int j = g; j < n; j += ng)
    for (int i = threadIdx.x % 64; i < n; i += 64) {
      const double w = W[(int64_t)j * ldw + i];
      const double d = w - (i == j ? 1.0 : 0.0);
      acc += d * d;
      acc2 += w * w;
    }
  red[threadIdx.x] = acc;
  red2[threadIdx.x] = acc2;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
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

size_t sketch_factor_scratch_doubles(int s, int n) {
  return (size_t)s * n + (size_t)32 * s + 32 * 32 + (size_t)n;
}

template <int NB, int RPL>
static hipError_t qr_blocked_t(int s, int n, const double* B, int64_t ldb, double* R,
                               int64_t ldr, int* info, double* scratch, hipStream_t st) {
  double* Wk = scratch;
  double* Vb = Wk + (size_t)s * n;
  double* Tb = Vb + (size_t)s * NB;
  double* betas = Tb + NB * NB;
  hipLaunchKernelGGL(k_copy_cols, dim3(n), dim3(256), 0, st, s, n, B, ldb, Wk);
  constexpr int kCpb = 8;  // trailing columns per update workgroup (one per wavefront)
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int w = (n - j0) < NB ? (n - j0) : NB;
    const int p = s - j0;
    hipLaunchKernelGGL((k_qr_panel<NB, RPL>), dim3(1), dim3(kSmallThreads),
                       qr_panel_lds_doubles<NB>(p) * sizeof(double), st, s, n, j0, Wk, Vb, Tb,
                       betas);
    const int rest = n - j0 - w;
    if (rest > 0)
      hipLaunchKernelGGL((k_qr_update<NB, RPL>), dim3((rest + kCpb - 1) / kCpb), dim3(512),
                         ((size_t)NB * p + NB * NB) * sizeof(double), st, s, n, j0, w, kCpb, Vb,
                         Tb, Wk);
  }
  hipLaunchKernelGGL(k_qr_finish, dim3(n), dim3(256), 0, st, s, n, Wk, betas, R, ldr, info);
  return hipGetLastError();
}

// Blocked Householder QR for s <= 2048; the panel width keeps a panel (and the update's
// copy of V) within 136 KiB of LDS.
static hipError_t launch_qr_blocked(int s, int n, const double* B, int64_t ldb, double* R,
                                    int64_t ldr, int* info, double* scratch, hipStream_t st) {
  if (s <= 512) return qr_blocked_t<32, 8>(s, n, B, ldb, R, ldr, info, scratch, st);
  if (s <= 1024) return qr_blocked_t<16, 16>(s, n, B, ldb, R, ldr, info, scratch, st);
  if (s <= 2048) return qr_blocked_t<8, 32>(s, n, B, ldb, R, ldr, info, scratch, st);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------------------
// Blocked partial-pivot LU of the s x n sketch (s <= 2048), in place in Wk (ld s):
//  (a) k_lu_panel: one workgroup factors columns j0 .. j0+nb-1 over rows j0 .. s-1, each
//      thread holding PR rows of the panel in registers (pivot = first largest |w_ik|, as
//      the unblocked kernels; two barriers per column), and records the pivots;
//  (b) k_lu_trail: one wavefront per trailing column applies the panel's row swaps in
//      order (lane j holds row j0 + j, and tracks the row its swap reaches below the
//      panel) and forms U12 = L11^{-1} A12 with the unit lower L11;
//  (c) k_lu_update: A22 -= L21 U12 (K = nb) over 16 x 16 output tiles staged in LDS.
// Only U is needed (R0 = diag(sign u_kk) U), so the swaps are not applied to L's columns.
// ------------------------------------------------------------------------------------
constexpr int kLuPanelThreads = 512;
constexpr int kLuPanelWaves = kLuPanelThreads / kWave;

template <int NB, int PR>  // panel rows s - j0 <= PR * kLuPanelThreads
__global__ __launch_bounds__(kLuPanelThreads) void k_lu_panel(int s, int n, int j0, double* Wk,
                                                              int* __restrict__ piv) {
  __shared__ double cand_v[kLuPanelWaves];
  __shared__ int cand_i[kLuPanelWaves];
  __shared__ double rowp[NB], rowk[NB];
  const int nb = min(NB, n - j0), rows = s - j0;
  const int t = (int)threadIdx.x, lane = lane_id(), wave = wave_id();
  double a[PR][NB];
#pragma unroll
  for (int u = 0; u < PR; ++u) {
    const int row = t + kLuPanelThreads * u;
    const bool rok = row < rows;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const bool ok = rok && c < nb;
      const double v = Wk[(int64_t)(j0 + (c < nb ? c : 0)) * s + j0 + (rok ? row : 0)];
      a[u][c] = ok ? v : 0.0;
    }
  }
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    if (k < nb) {  // uniform (a guard, not a break: the panel stays in registers)
    double bv = -1.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int u = 0; u < PR; ++u) {
      const int row = t + kLuPanelThreads * u;
      const double av = fabs(a[u][k]);
      if (row >= k && row < rows && piv_better(av, row, bv, bi)) {
        bv = av;
        bi = row;
      }
    }
    wave_argmax(bv, bi);
    if (lane == 0) {
      cand_v[wave] = bv;
      cand_i[wave] = bi;
    }
    __syncthreads();
    // every thread combines the candidates (a total order: the same p everywhere)
    double pv = cand_v[0];
    int p = cand_i[0];
#pragma unroll
    for (int w = 1; w < kLuPanelWaves; ++w) {
      const double cv = cand_v[w];
      const int ci = cand_i[w];
      if (piv_better(cv, ci, pv, p)) {
        pv = cv;
        p = ci;
      }
    }
    // publish rows p and k (before the swap)
#pragma unroll
    for (int u = 0; u < PR; ++u) {
      const int row = t + kLuPanelThreads * u;
      if (row == p)
#pragma unroll
        for (int c = 0; c < NB; ++c) rowp[c] = a[u][c];
      if (row == k)
#pragma unroll
        for (int c = 0; c < NB; ++c) rowk[c] = a[u][c];
    }
    __syncthreads();
    const double pivot = rowp[k];
#pragma unroll
    for (int u = 0; u < PR; ++u) {
      const int row = t + kLuPanelThreads * u;
      const bool isk = row == k, isp = row == p && p != k, below = row > k && row < rows;
      double x[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) x[c] = isk ? rowp[c] : (isp ? rowk[c] : a[u][c]);
      const double l = x[k] / pivot;
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c == k) a[u][c] = below ? l : x[c];
        else if (c > k) a[u][c] = below ? x[c] - l * rowp[c] : x[c];
        else a[u][c] = x[c];
      }
    }
    if (t == 0) piv[j0 + k] = j0 + p;
    }
  }
#pragma unroll
  for (int u = 0; u < PR; ++u) {
    const int row = t + kLuPanelThreads * u;
    if (row < rows)
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nb) Wk[(int64_t)(j0 + c) * s + j0 + row] = a[u][c];
  }
}

template <int NB>
__global__ __launch_bounds__(256) void k_lu_trail(int s, int n, int j0, int nb, double* Wk,
                                                  const int* __restrict__ piv) {
  const int lane = lane_id(), wave = wave_id();
  const int c = j0 + nb + 4 * (int)blockIdx.x + wave;
  if (c >= n) return;
  double* col = Wk + (int64_t)c * s;
  const bool in = lane < nb;
  const int pj = in ? piv[j0 + lane] : j0;  // lane j: the row swapped with row j0 + j
  const bool below = in && pj >= j0 + nb;
  double x = col[j0 + (in ? lane : 0)];
  double xb = col[below ? pj : j0];          // lane j: the current value of row pj
  // L11 row of this lane (columns l < lane), loaded while the swaps run
  double lrow[NB];
#pragma unroll
  for (int l = 0; l < NB; ++l) lrow[l] = Wk[(int64_t)(j0 + (l < nb ? l : 0)) * s + j0 + (in ? lane : 0)];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int p = __builtin_amdgcn_readlane(pj, j);
    if (j < nb && p != j0 + j) {
      const double xj = readlane_f64(x, j);
      if (p < j0 + nb) {
        const double xp = readlane_f64(x, p - j0);
        x = (lane == j) ? xp : ((lane == p - j0) ? xj : x);
      } else {
        const double xp = readlane_f64(xb, j);  // lane j tracks row p
        x = (lane == j) ? xp : x;
        xb = (below && pj == p) ? xj : xb;
      }
    }
  }
  // forward substitution with the unit lower L11
#pragma unroll
  for (int l = 0; l < NB; ++l) {
    const double xl = readlane_f64(x, l);
    x -= (in && lane > l && l < nb) ? lrow[l] * xl : 0.0;
  }
  if (in) col[j0 + lane] = x;
  if (below) col[pj] = xb;
}

__global__ __launch_bounds__(256) void k_lu_update(int s, int n, int j0, int nb, double* Wk) {
  __shared__ double Ls[16][33], Us[32][17];
  const int i0 = j0 + nb + 16 * blockIdx.y, c0 = j0 + nb + 16 * blockIdx.x;
  const int ti = threadIdx.x % 16, tc = threadIdx.x / 16;
  for (int e = threadIdx.x; e < 16 * nb; e += 256) {
    const int r = e % 16, k = e / 16;
    Ls[r][k] = (i0 + r < s) ? Wk[(int64_t)(j0 + k) * s + i0 + r] : 0.0;
    const int kk = e % nb, cc = e / nb;
    Us[kk][cc] = (c0 + cc < n) ? Wk[(int64_t)(c0 + cc) * s + j0 + kk] : 0.0;
  }
  __syncthreads();
  const int i = i0 + ti, c = c0 + tc;
  if (i < s && c < n) {
    double acc = 0.0;
    for (int k = 0; k < nb; ++k) acc += Ls[ti][k] * Us[k][tc];
    Wk[(int64_t)c * s + i] -= acc;
  }
}

// R = diag(sign u_kk) U from the factored Wk; a zero or NaN u_kk at the first such k sets
// *info = 1000 + k + 1 (if it was 0) and R(k, k) = NaN.
__global__ __launch_bounds__(256) void k_lu_finish(int s, int n, const double* __restrict__ Wk,
                                                   double* __restrict__ R, int64_t ldr,
                                                   int* __restrict__ info) {
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = 0.0;
    if (i <= c) {
      const double ui = Wk[(int64_t)i * s + i];
      const double sg = (ui < 0.0) ? -1.0 : 1.0;
      v = (i == c) ? fabs(ui) : sg * Wk[(int64_t)c * s + i];
      if (i == c && !(ui != 0.0)) v = NAN;
    }
    R[(int64_t)c * ldr + i] = v;
  }
  if (c == 0 && info) {
    const int bad = block_first_bad(n, [&](int k) { return Wk[(int64_t)k * s + k]; });
    if (threadIdx.x == 0 && bad && *info == 0) *info = 1000 + bad;
  }
}

template <int NB, int PR>
static hipError_t lu_blocked_t(int s, int n, const double* B, int64_t ldb, double* R,
                               int64_t ldr, int* info, double* scratch, hipStream_t st) {
  static_assert(NB <= kWave, "k_lu_trail holds the panel's rows in one wavefront's lanes");
  if (s > PR * kLuPanelThreads || n > s) return hipErrorInvalidValue;  // panel rows per thread
  double* Wk = scratch;
  int* piv = reinterpret_cast<int*>(scratch + (size_t)s * n);
  hipLaunchKernelGGL(k_copy_cols, dim3(n), dim3(256), 0, st, s, n, B, ldb, Wk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int nb = NB < n - j0 ? NB : n - j0;
    hipLaunchKernelGGL((k_lu_panel<NB, PR>), dim3(1), dim3(kLuPanelThreads), 0, st, s, n, j0, Wk,
                       piv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int t = n - j0 - nb;
    if (t > 0) {
      hipLaunchKernelGGL(k_lu_trail<NB>, dim3((t + 3) / 4), dim3(256), 0, st, s, n, j0, nb, Wk,
                         piv);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const int rows = s - j0 - nb;
      hipLaunchKernelGGL(k_lu_update, dim3((t + 15) / 16, (rows + 15) / 16), dim3(256), 0, st, s,
                         n, j0, nb, Wk);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(k_lu_finish, dim3(n), dim3(256), 0, st, s, n, Wk, R, ldr, info);
  return hipGetLastError();
}

hipError_t launch_sketch_factor(int variant, int s, int n, const double* B, int64_t ldb,
                                double* R, int64_t ldr, int* info, double* scratch,
                                hipStream_t st) {
  const int rpl = pow2_at_least((s + 63) / 64), cpw = pow2_at_least((n + 15) / 16);
  dim3 grid(1), block(kSmallThreads);
  // LU with implicit interchanges from two rows per lane up to 256 rows, 33..128 columns
  // (measured against the blocked form: 256 x 128, 360 -> 325 us; 256 x 64, 184 -> 127 us;
  // 128 x 64, 180 -> 88 us)
  if (variant == 1 && (rpl == 2 || rpl == 4) && (cpw == 4 || cpw == 8)) {
    if (rpl == 2 && cpw == 4)
      hipLaunchKernelGGL((k_getrf_ip<2, 4>), grid, block, 0, st, s, n, B, ldb, R, ldr, info);
    else if (rpl == 2)
      hipLaunchKernelGGL((k_getrf_ip<2, 8>), grid, block, 0, st, s, n, B, ldb, R, ldr, info);
    else if (cpw == 4)
      hipLaunchKernelGGL((k_getrf_ip<4, 4>), grid, block, 0, st, s, n, B, ldb, R, ldr, info);
    else
      hipLaunchKernelGGL((k_getrf_ip<4, 8>), grid, block, 0, st, s, n, B, ldb, R, ldr, info);
    return hipGetLastError();
  }
  // LU of 64+ columns over 257..512 rows: the blocked form (it was faster than the
  // explicit-interchange register kernel from n = 64: 256 x 128, 0.40 -> 0.38 ms)
  if (variant == 1 && n >= 64 && s <= 512)
    return lu_blocked_t<16, 1>(s, n, B, ldb, R, ldr, info, scratch, st);
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
  if (variant == 0 && s <= 2048) return launch_qr_blocked(s, n, B, ldb, R, ldr, info, scratch, st);
  // panel registers per thread: NB x PR <= 32 doubles
  if (variant == 1 && s <= 512) return lu_blocked_t<16, 1>(s, n, B, ldb, R, ldr, info, scratch, st);
  if (variant == 1 && s <= 1024) return lu_blocked_t<16, 2>(s, n, B, ldb, R, ldr, info, scratch, st);
  if (variant == 1 && s <= 2048) return lu_blocked_t<8, 4>(s, n, B, ldb, R, ldr, info, scratch, st);
  if (variant == 1) {
    const size_t sh = (size_t)(2 * s + n) * sizeof(double) + 2 * sizeof(int);
    hipLaunchKernelGGL(k_getrf_glb, grid, block, sh, st, s, n, B, ldb, R, ldr, info, scratch);
  } else {
    const size_t sh = (size_t)(2 * s + 2 + n) * sizeof(double);
    hipLaunchKernelGGL(k_geqrf_glb, grid, block, sh, st, s, n, B, ldb, R, ldr, info, scratch);
  }
  return hipGetLastError();
}

#ifndef TSQR_POTRF_MULTI_NB
#define TSQR_POTRF_MULTI_NB 32
#endif
constexpr int kPotrfMultiNB = TSQR_POTRF_MULTI_NB;  // n > kCholLdsMax: one launch per phase

hipError_t launch_potrf(int n, const double* W, int64_t ldw, double* R, int64_t ldr, int stage,
                        int* info, double* scratch, hipStream_t st, double shift,
                        const int* gate) {
  (void)scratch;
  if (n < 1 || n > kMaxS) return hipErrorInvalidValue;
  // one workgroup with the matrix in LDS up to 128 columns (measured against the
  // column-at-a-time register factorization, one barrier per column, that the batched
  // kernels use: n = 32, 13.4 -> 10.8 us; n = 64, 33.5 -> 21.5 us; n = 128, 144 -> 49 us)
  if (n <= kCholLdsMax) {
    hipLaunchKernelGGL(k_potrf_lds, dim3(1), dim3(kSmallThreads), chol_lds_bytes(n), st, n, W,
                       ldw, R, ldr, stage, info, shift, gate);
    return hipGetLastError();
  }
  return potrf_multi_t<kPotrfMultiNB>(n, W, ldw, R, ldr, stage, info, st, shift, gate);
}

hipError_t launch_trmm_upper(int n, const double* A, int64_t lda, const double* B, int64_t ldb,
                             double* C, int64_t ldc, hipStream_t st, const int* gate) {
  const int nb = (n + 15) / 16;
  hipLaunchKernelGGL(k_trmm_upper, dim3(nb, nb), dim3(256), 0, st, n, A, lda, B, ldb, C, ldc,
                     gate);
  return hipGetLastError();
}

hipError_t launch_poison(const int* info, int64_t m, int n, double* Q, int64_t ldq, double* R,
                         int64_t ldr, hipStream_t st) {
  // grid-strided fill: a small grid costs little when nothing broke down (the usual case)
  hipLaunchKernelGGL(k_poison, dim3(256), dim3(256), 0, st, info, m, n, Q, ldq, R, ldr);
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

// W(k, k) += coef * (*scale) (or coef when scale is null): the diagonal shift of the first
// Gram matrix in shifted CholeskyQR, with the scale read on the device (no host wait).
__global__ __launch_bounds__(256) void k_add_diag(int n, double* __restrict__ W, int64_t ldw,
                                                  double coef, const double* __restrict__ scale,
                                                  const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  const double sh = scale ? coef * *scale : coef;
  for (int k = threadIdx.x + blockIdx.x * blockDim.x; k < n; k += blockDim.x * gridDim.x)
    W[(int64_t)k * ldw + k] += sh;
}

hipError_t launch_add_diag(int n, double* W, int64_t ldw, double coef, const double* scale,
                           hipStream_t st, const int* gate) {
  hipLaunchKernelGGL(k_add_diag, dim3((n + 255) / 256), dim3(256), 0, st, n, W, ldw, coef, scale,
                     gate);
  return hipGetLastError();
}

hipError_t launch_pass_decide(int n, const double* W, int64_t ldw, const int* lp_info,
                              const int* info, double thresh, int* need, double* dev_out,
                              hipStream_t st, const int* gate) {
  hipLaunchKernelGGL(k_pass_decide, dim3(1), dim3(1024), 0, st, n, W, ldw, lp_info, info, thresh,
                     need, dev_out, gate);
  return hipGetLastError();
}

// ---- decisions of the mixed-precision chain (one thread) ---------------------------------
__global__ void k_mixed_ctl(int op, int k, int arg, double arg2, MixedCtl* __restrict__ c,
                            int* __restrict__ info, int* __restrict__ d_passes) {
  switch (op) {
    case kCtlInit:
      c->stage = 1;
      c->lp_info = 0;
      for (int p = 0; p <= kMaxMixedPasses; ++p) c->gate[p] = arg > 0 ? (p < arg) : (p == 0);
      for (int p = 0; p < kMaxMixedPasses; ++p) {
        c->skip[p] = 0;
        c->bd[p] = 0;
        c->shifted[p] = 0;
      }
      c->one = 1;
      c->passes = 0;
      break;
    case kCtlStage:
      c->stage = (c->norms[1] * c->norms[3] * arg2 <= 1.0) ? 1 : 0;
      c->lp_info = c->stage ? 0 : -1;
      break;
    case kCtlPassBegin:
      c->bd[k] = 0;
      c->skip[k] = c->gate[k] ? 0 : 1;
      break;
    case kCtlShift:
      c->shifted[k] = (c->gate[k] && c->bd[k] != 0) ? 1 : 0;
      break;
    case kCtlNext:
      // another pass while this pass needed the shift or its input's Gram matrix deviated
      // from I by more than arg2 (NaN counts as deviating)
      c->gate[k + 1] = (k + 1 < arg && c->gate[k] &&
                        (c->shifted[k] || !(c->dev[k][0] <= arg2))) ? 1 : 0;
      break;
    case kCtlEnd: {
      int p = 0;
      for (int q = 0; q < kMaxMixedPasses; ++q) p += c->gate[q];
      c->passes = p;
      if (p == arg && arg > 0 && c->shifted[arg - 1] && info && *info == 0) *info = 5000;
      if (d_passes) {
        d_passes[0] = p;
        d_passes[1] = c->stage;
      }
      break;
    }
    default:
      break;
  }
}

hipError_t launch_mixed_ctl(int op, int k, int arg, double arg2, MixedCtl* c, int* info,
                            int* d_passes, hipStream_t st) {
  hipLaunchKernelGGL(k_mixed_ctl, dim3(1), dim3(1), 0, st, op, k, arg, arg2, c, info, d_passes);
  return hipGetLastError();
}

// ---- batched forms ----------------------------------------------------------------------
template <int RPL, int CPW>
__global__ __launch_bounds__(kSmallThreads) void k_b_geqrf(const BItem* __restrict__ items,
                                                           const BProb* __restrict__ probs) {
  const BProb& p = probs[items[blockIdx.x].pid];
  geqrf_reg_body<RPL, CPW, false, RPL >= 2 && (CPW == 8 || CPW == 4)>(p.s, p.n, p.B, p.s,
                                                                      p.R0, p.n, p.info);
}

template <int RPL, int CPW>
__global__ __launch_bounds__(kSmallThreads) void k_b_getrf(const BItem* __restrict__ items,
                                                           const BProb* __restrict__ probs) {
  const BProb& p = probs[items[blockIdx.x].pid];
  getrf_reg_body<RPL, CPW>(p.s, p.n, p.B, p.s, p.R0, p.n, p.info);
}

template <int RPL, int CPW>
__global__ __launch_bounds__(kSmallThreads) void k_b_potrf(int which, int stage,
                                                           const BItem* __restrict__ items,
                                                           const BProb* __restrict__ probs) {
  const BProb& p = probs[items[blockIdx.x].pid];
  potrf_reg_body<RPL, CPW>(p.n, p.W, p.n, which == 1 ? p.R1 : p.R2, p.n, stage, p.info, 0.0);
}

__global__ __launch_bounds__(256) void k_b_trmm(int which, const BItem* __restrict__ items,
                                                const BProb* __restrict__ probs) {
  const BItem it = items[blockIdx.x];
  const BProb& p = probs[it.pid];
  if (which == 0)
    trmm_upper_body(p.n, p.R1, p.n, p.R0, p.n, p.R10, p.n, it.x, it.y);
  else if (p.R)
    trmm_upper_body(p.n, p.R2, p.n, p.R10, p.n, p.R, p.ldr, it.x, it.y);
}

__global__ __launch_bounds__(256) void k_b_poison(const BItem* __restrict__ items,
                                                  const BProb* __restrict__ probs) {
  const BItem it = items[blockIdx.x];
  const BProb& p = probs[it.pid];
  poison_body(p.info, p.m, p.n, p.Q, p.ldq, p.R, p.ldr, it.x, p.poison_wgs);
}

__global__ void k_b_set_info(const BItem* __restrict__ items, const BProb* __restrict__ probs) {
  if (threadIdx.x == 0) *probs[items[blockIdx.x].pid].info = 0;
}

hipError_t launch_b_factor(int variant, int RPL, int CPW, const BItem* items, int nitems,
                           const BProb* probs, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
#define TSQR_BF(RPL_, CPW_)                                                                   \
  if (RPL == RPL_ && CPW == CPW_) {                                                           \
    if (variant == 1)                                                                         \
      hipLaunchKernelGGL((k_b_getrf<RPL_, CPW_>), dim3(nitems), dim3(kSmallThreads), 0, st,    \
                         items, probs);                                                       \
    else                                                                                      \
      hipLaunchKernelGGL((k_b_geqrf<RPL_, CPW_>), dim3(nitems), dim3(kSmallThreads), 0, st,    \
                         items, probs);                                                       \
    return hipGetLastError();                                                                 \
  }
  TSQR_BF(1, 1) TSQR_BF(1, 2) TSQR_BF(1, 4) TSQR_BF(1, 8)
  TSQR_BF(2, 1) TSQR_BF(2, 2) TSQR_BF(2, 4) TSQR_BF(2, 8)
  TSQR_BF(4, 1) TSQR_BF(4, 2) TSQR_BF(4, 4) TSQR_BF(4, 8)
  TSQR_BF(8, 1) TSQR_BF(8, 2) TSQR_BF(8, 4)
#undef TSQR_BF
  return hipErrorInvalidValue;
}

hipError_t launch_b_potrf(int RPL, int CPW, int which, int stage, const BItem* items,
                          int nitems, const BProb* probs, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
#define TSQR_BP(RPL_, CPW_)                                                                   \
  if (RPL == RPL_ && CPW == CPW_) {                                                           \
    hipLaunchKernelGGL((k_b_potrf<RPL_, CPW_>), dim3(nitems), dim3(kSmallThreads), 0, st,      \
                       which, stage, items, probs);                                           \
    return hipGetLastError();                                                                 \
  }
  TSQR_BP(1, 1) TSQR_BP(1, 2) TSQR_BP(1, 4) TSQR_BP(2, 8)
#undef TSQR_BP
  return hipErrorInvalidValue;
}

hipError_t launch_b_trmm(int which, const BItem* items, int nitems, const BProb* probs,
                         hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_trmm, dim3(nitems), dim3(256), 0, st, which, items, probs);
  return hipGetLastError();
}

hipError_t launch_b_poison(const BItem* items, int nitems, const BProb* probs, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_poison, dim3(nitems), dim3(256), 0, st, items, probs);
  return hipGetLastError();
}

hipError_t launch_b_set_info(const BItem* items, int nitems, const BProb* probs, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_set_info, dim3(nitems), dim3(64), 0, st, items, probs);
  return hipGetLastError();
}

}  // namespace tsqr
