// Tall-skinny kernels of CholeskyQR (paper Algorithm CholeskyQR): the right-side
// triangular solve X = Y T^{-1} and the Gram matrix W = X^T X, both on FP64 MFMA.
#include "tsqr_device.hpp"
#include "tsqr_launch.hpp"

namespace tsqr {

// ------------------------------------------------------------------------------------
// X = Y T^{-1}, T upper triangular (n x n): blocked substitution over 16-column blocks,
// entirely on FP64 MFMA, in the transposed form
//   X_b^T = T_bb^{-T} (Y_b^T - sum_{a<b} T_ab^T X_a^T).
// Register layout (one wavefront per 16-row tile): lane l (group q = l/16, row c = l%16)
// holds columns 16b + 4q + r (r = 0..3) of every block b.  The MFMA accumulator of a block
// is X_b^T with its 16 rows permuted by sigma(4r + q) = 4q + r (the A operand of lane l
// reads column sigma(l%16) of its T tile), so accumulator register kk is exactly the B
// operand of K-step kk (MFMA k-index q <-> column 16b + 4q + kk): solved blocks feed the
// updates of later blocks without any data movement.
// Diagonal blocks: X0 = C T_bb^{-1} with the explicitly inverted 16x16 block, followed
// (when the block's infinity-norm condition estimate exceeds 16) by one correction step
// E = C - X0 T_bb, X = X0 + E T_bb^{-1}.  The correction removes the cond(T_bb) factor
// from the error of multiplying by an inverse, so each row keeps the backward error of
// substitution (|Y - X T| ~ n u |X||T|) even for the ill-conditioned R0 of the sketch.
// Operand tiles are prepared once per solve by k_trsm_prep (negated, sigma-permuted).
// Rows >= m are zero and never stored; columns >= n see T padded with the identity.
// X may alias Y: each wavefront reads its whole tile before writing it.
// ------------------------------------------------------------------------------------
__host__ __device__ constexpr int tri_a(int t) {
  int b = 0;
  while ((b + 1) * (b + 2) / 2 <= t) ++b;
  return t - b * (b + 1) / 2;
}
__host__ __device__ constexpr int tri_b(int t) {
  int b = 0;
  while ((b + 1) * (b + 2) / 2 <= t) ++b;
  return b;
}
__host__ __device__ constexpr int sigma16(int x) { return 4 * (x & 3) + (x >> 2); }
__host__ __device__ constexpr int off_index(int a, int b) { return b * (b - 1) / 2 + a; }

typedef __attribute__((address_space(3))) double lds_f64;

// Prepared operand buffer, tiles of 256 doubles stored as tile[i*16 + sigma16(j)]:
//   [0, NOFF)          off-diagonal tiles (a < b): -T(16a+i, 16b+j)
//   [NOFF, NOFF+JT)    diagonal tiles: -T(16b+i, 16b+j) for i <= j, else 0
//   [NOFF+JT, +2JT)    inverted diagonal tiles: (T_bb^{-1})(i, j)
// then JT ints: 1 if the block needs the correction step.
constexpr double kTrsmRefineCond = 16.0;

__host__ __device__ constexpr size_t trsm_prep_doubles(int jt) {
  return (size_t)(jt * (jt - 1) / 2 + 2 * jt) * 256 + (size_t)(jt + 1) / 2 + 1;
}

__global__ __launch_bounds__(256) void k_trsm_prep(int n, int jt, const double* __restrict__ T,
                                                   int64_t ldt, double* __restrict__ P) {
  const int b = blockIdx.x;  // block column handled by this workgroup
  const int noff = jt * (jt - 1) / 2;
  auto Tg = [&](int i, int j) -> double {
    return (i < n && j < n) ? T[(int64_t)j * ldt + i] : (i == j ? 1.0 : 0.0);
  };
  for (int a = 0; a < b; ++a)
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
      const int i = e / 16, j = e % 16;
      P[(size_t)off_index(a, b) * 256 + i * 16 + sigma16(j)] = -Tg(16 * a + i, 16 * b + j);
    }
  __shared__ double tb[16][17];
  __shared__ double ti[16][17];
  for (int e = threadIdx.x; e < 256; e += blockDim.x) {
    const int i = e / 16, j = e % 16;
    const double v = (i <= j) ? Tg(16 * b + i, 16 * b + j) : 0.0;
    tb[i][j] = v;
    P[(size_t)(noff + b) * 256 + i * 16 + sigma16(j)] = -v;
  }
  __syncthreads();
  if (threadIdx.x < 16) {  // column j of the inverse by back substitution
    const int j = threadIdx.x;
    for (int i = 15; i >= 0; --i) {
      double acc = (i == j) ? 1.0 : 0.0;
      for (int k = i + 1; k <= j; ++k) acc -= tb[i][k] * ti[k][j];
      ti[i][j] = (i <= j) ? acc / tb[i][i] : 0.0;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 256; e += blockDim.x) {
    const int i = e / 16, j = e % 16;
    P[(size_t)(noff + jt + b) * 256 + i * 16 + sigma16(j)] = ti[i][j];
  }
  if (threadIdx.x == 0) {  // infinity-norm condition estimate of the block
    double nt = 0.0, ni = 0.0;
    for (int i = 0; i < 16; ++i) {
      double st = 0.0, si = 0.0;
      for (int j = 0; j < 16; ++j) {
        st += fabs(tb[i][j]);
        si += fabs(ti[i][j]);
      }
      nt = fmax(nt, st);
      ni = fmax(ni, si);
    }
    const double c = nt * ni;
    int* flags = reinterpret_cast<int*>(P + (size_t)(noff + 2 * jt) * 256);
    flags[b] = (c > kTrsmRefineCond || !(c == c)) ? 1 : 0;
  }
}

template <int JT, bool kLds>
__global__ __launch_bounds__(512, 1) void k_trsm_mfma(int64_t m, int n,
                                                      const double* __restrict__ Y, int64_t ldy,
                                                      const double* __restrict__ P,
                                                      double* X, int64_t ldx) {
  constexpr int NOFF = JT * (JT - 1) / 2;
  constexpr int NTILE = NOFF + 2 * JT;
  extern __shared__ double tl[];
  const int* flags_g = reinterpret_cast<const int*>(P + (size_t)NTILE * 256);
  __shared__ int flags[JT];
  if (kLds)
    for (int e = threadIdx.x; e < NTILE * 256; e += blockDim.x) tl[e] = P[e];
  for (int e = threadIdx.x; e < JT; e += blockDim.x) flags[e] = flags_g[e];
  __syncthreads();

  const int lane = lane_id();
  const int q = lane >> 4, c16 = lane & 15;
  const int64_t ntiles = (m + 15) / 16;
  const int nw = blockDim.x / kWave;
  const int64_t wstride = (int64_t)gridDim.x * nw;
  for (int64_t tile = (int64_t)blockIdx.x * nw + wave_id(); tile < ntiles; tile += wstride) {
    // opaque per-iteration bases: the tiles are loop invariant and would otherwise be
    // hoisted into registers
    lds_f64* tlp = (lds_f64*)tl;
    const double* Pg = P;
    asm volatile("" : "+v"(tlp), "+s"(Pg));
    auto Aop = [&](int t, int kk) -> double {
      const int o = t * 256 + (4 * q + kk) * 16 + c16;
      return kLds ? tlp[o] : Pg[o];
    };
    const int64_t row = tile * 16 + c16;
    const bool rok = row < m;
    v4d xr[JT];
#pragma unroll
    for (int b = 0; b < JT; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = 16 * b + 4 * q + r;
        xr[b][r] = (rok && col < n) ? Y[(int64_t)col * ldy + row] : 0.0;
      }

#pragma unroll
    for (int b = 0; b < JT; ++b) {
      // diagonal block: X0 = C T^{-1}, optional correction X = X0 + (C - X0 T) T^{-1}
      const v4d C = xr[b];
      v4d x0 = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) x0 = mfma_f64(Aop(NOFF + JT + b, kk), C[kk], x0);
      if (flags[b]) {
        v4d e = C;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) e = mfma_f64(Aop(NOFF + b, kk), x0[kk], e);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) x0 = mfma_f64(Aop(NOFF + JT + b, kk), e[kk], x0);
      }
      xr[b] = x0;
      // right-looking update of the later blocks
#pragma unroll
      for (int bb = b + 1; bb < JT; ++bb)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
          xr[bb] = mfma_f64(Aop(off_index(b, bb), kk), xr[b][kk], xr[bb]);
    }

    if (rok) {
#pragma unroll
      for (int b = 0; b < JT; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int col = 16 * b + 4 * q + r;
          if (col < n) X[(int64_t)col * ldx + row] = xr[b][r];
        }
    }
  }
}

size_t trsm_scratch_doubles(int n) {
  int jt = 1;
  while (jt < (n + 15) / 16) jt <<= 1;
  return trsm_prep_doubles(jt);
}

hipError_t launch_trsm(int64_t m, int n, const double* Y, int64_t ldy, const double* T,
                       int64_t ldt, double* X, int64_t ldx, double* scratch, hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  int jt = 1;
  while (jt < (n + 15) / 16) jt <<= 1;
  if (jt > 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trsm_prep, dim3(jt), dim3(256), 0, st, n, jt, T, ldt, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t ntiles = (m + 15) / 16;
  int64_t blocks = (ntiles + 7) / 8;
  const int64_t cap = (int64_t)device_cu_count();
  if (blocks > cap) blocks = cap;
  dim3 grid((unsigned)blocks), block(512);
#define TSQR_TRSM(J, L)                                                                    \
  if (jt == J) {                                                                           \
    const size_t sh = L ? (size_t)(J * (J - 1) / 2 + 2 * J) * 256 * sizeof(double) : 0;    \
    hipLaunchKernelGGL((k_trsm_mfma<J, L>), grid, block, sh, st, m, n, Y, ldy, scratch, X, \
                       ldx);                                                               \
    return hipGetLastError();                                                              \
  }
  TSQR_TRSM(1, true) TSQR_TRSM(2, true) TSQR_TRSM(4, true) TSQR_TRSM(8, true)
  TSQR_TRSM(16, false)
#undef TSQR_TRSM
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------------------
// Gram matrix W = X^T X (upper 16x16 tiles), split over row blocks.  A workgroup stages
// 64 rows of X in LDS (row-major, padded) and each wavefront accumulates a fixed subset
// of the upper tiles; for MFMA K-step kk, lane l reads X(row 4kk + l/16, col 16c + l%16),
// which is simultaneously the A operand (X^T) of tile (c, .) and the B operand of (., c).
// Partials are written tile-natively and summed in a fixed order by k_gram_reduce.
// ------------------------------------------------------------------------------------
template <int JT, int NW>
__global__ __launch_bounds__(NW * 64) void k_gram_f64(int64_t m, int n,
                                                      const double* __restrict__ X, int64_t ldx,
                                                      int64_t rows_per_block, int ntiles,
                                                      double* __restrict__ part) {
  constexpr int KC = 64;
  constexpr int NC = JT * 16;
  constexpr int LDN = NC + 1;
  constexpr int NT = JT * (JT + 1) / 2;
  constexpr int TPW = (NT + NW - 1) / NW;
  constexpr int THREADS = NW * 64;
  __shared__ double lds[KC * LDN];

  const int lane = lane_id(), wave = wave_id();
  const int q = lane >> 4, c16 = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(m, r0 + rows_per_block);

  v4d acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};

  for (int64_t rb = r0; rb < r1; rb += KC) {
    __syncthreads();
    // col-major global (rows contiguous) -> row-major LDS
    for (int e = threadIdx.x; e < KC * NC; e += THREADS) {
      const int rr = e % KC, cc = e / KC;
      const int64_t row = rb + rr;
      lds[rr * LDN + cc] = (row < r1 && cc < n) ? X[(int64_t)cc * ldx + row] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC / 4; ++kk) {
      double op[JT];
#pragma unroll
      for (int c = 0; c < JT; ++c) op[c] = lds[(4 * kk + q) * LDN + 16 * c + c16];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        if (t % NW == wave) acc[t / NW] = mfma_f64(op[tri_a(t)], op[tri_b(t)], acc[t / NW]);
      }
    }
  }

  // tiles are enumerated column by column, so the first `ntiles` are those of the
  // n x n matrix (the rest only exist in the padded template size)
  double* dst = part + (size_t)blockIdx.x * ntiles * 256;
#pragma unroll
  for (int t = 0; t < NT; ++t)
    if (t % NW == wave && t < ntiles)
      *reinterpret_cast<v4d*>(dst + (size_t)t * 256 + lane * 4) = acc[t / NW];
}

// W(i, j) = W(j, i) = sum_kb part[kb][tile][lane][reg]; same deterministic two-level
// order as the sketch reduction (16 strided groups, then the groups in order).
__global__ __launch_bounds__(256) void k_gram_reduce(int kblocks, int ntiles, int n,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ W, int64_t ldw) {
  __shared__ double red[16][17];
  const size_t E = (size_t)ntiles * 256;
  const int g = threadIdx.x / 16, o = threadIdx.x % 16;
  const size_t e = (size_t)blockIdx.x * 16 + o;
  double acc = 0.0;
  if (e < E)
    for (int kb = g; kb < kblocks; kb += 16) acc += part[(size_t)kb * E + e];
  red[g][o] = acc;
  __syncthreads();
  if (g == 0 && e < E) {
    double t = 0.0;
    for (int k = 0; k < 16; ++k) t += red[k][o];
    const int tile = (int)(e / 256), lane = (int)((e / 4) % 64), r = (int)(e % 4);
    const int a = tri_a(tile), b = tri_b(tile);
    const int i = 16 * a + 4 * r + (lane >> 4), j = 16 * b + (lane & 15);
    if (i < n && j < n) {
      W[(int64_t)j * ldw + i] = t;
      W[(int64_t)i * ldw + j] = t;
    }
  }
}

GramPlan plan_gram(int64_t m, int n) {
  GramPlan p{};
  p.jt_total = (n + 15) / 16;
  p.ntiles = p.jt_total * (p.jt_total + 1) / 2;
  const int64_t target = (int64_t)device_cu_count() * 2;
  int64_t rpb = (m + target - 1) / target;
  rpb = ((rpb + 63) / 64) * 64;
  if (rpb < 64) rpb = 64;
  p.rows_per_block = rpb;
  p.kblocks = (int)((m + rpb - 1) / rpb);
  if (p.kblocks < 1) p.kblocks = 1;
  p.part_doubles = (size_t)p.kblocks * p.ntiles * 256;
  return p;
}

hipError_t launch_gram(const GramPlan& p, int64_t m, int n, const double* X, int64_t ldx,
                       double* part, hipStream_t st) {
  dim3 grid(p.kblocks);
#define TSQR_GRAM(J, NW_)                                                                   \
  if (p.jt_total <= J) {                                                                   \
    hipLaunchKernelGGL((k_gram_f64<J, NW_>), grid, dim3(NW_ * 64), 0, st, m, n, X, ldx,     \
                       p.rows_per_block, p.ntiles, part);                                             \
    return hipGetLastError();                                                               \
  }
  TSQR_GRAM(1, 4) TSQR_GRAM(2, 4) TSQR_GRAM(4, 4) TSQR_GRAM(8, 4) TSQR_GRAM(16, 8)
#undef TSQR_GRAM
  return hipErrorInvalidValue;
}

hipError_t launch_gram_reduce(const GramPlan& p, int n, const double* part, double* W,
                              int64_t ldw, hipStream_t st) {
  const size_t E = (size_t)p.ntiles * 256;
  const int blocks = (int)((E + 15) / 16);
  hipLaunchKernelGGL(k_gram_reduce, dim3(blocks), dim3(256), 0, st, p.kblocks, p.ntiles, n, part,
                     W, ldw);
  return hipGetLastError();
}

}  // namespace tsqr
