// Tall-skinny kernels of CholeskyQR (paper Algorithm CholeskyQR): the right-side
// triangular solve X = Y T^{-1} and the Gram matrix W = X^T X, both on FP64 MFMA.
#include "tsqr_device.hpp"
#include "tsqr_launch.hpp"

namespace tsqr {

// ------------------------------------------------------------------------------------
// X = Y T^{-1}, T upper triangular (n x n).  One wavefront solves a 16-row tile by
// blocked substitution over 16-column blocks, in the transposed form
//   X_b^T = T_bb^{-T} (Y_b^T - sum_{a<b} T_ab^T X_a^T):
//   * lane l (group q = l/16, row c = l%16 of the tile) holds columns 16b + 4q + r,
//     r = 0..3, of every block b: a contiguous quad of columns per lane group;
//   * the accumulator of the MFMA update of block bb is X_bb^T with its 16 rows permuted
//     by sigma(4r + q) = 4q + r (the A operand of lane l reads T column sigma(l%16)), so the
//     accumulator registers are exactly the quads above, and register kk of block b is the
//     B operand of K-step kk (MFMA k-index q <-> column 16b + 4q + kk): solved values feed
//     the updates without data movement;
//   * the 16x16 diagonal blocks are solved by substitution (row-wise backward stable, no
//     explicit inverse): each lane group solves its own quad locally, then broadcasts
//     the four solved values of the row to the later groups (one shuffle round per quad);
//   * right-looking order: a solved block immediately updates every later block.
// Columns >= n and rows >= m are padded (T as identity, Y as zero) and never stored.
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
__host__ __device__ constexpr int tri_index(int a, int b) { return b * (b + 1) / 2 + a; }
__host__ __device__ constexpr int sigma16(int x) { return 4 * (x & 3) + (x >> 2); }

typedef __attribute__((address_space(3))) double lds_f64;

// T staged in LDS as its upper 16x16 tiles (tile-major, row-major inside a tile): the
// off-diagonal tiles negated and with columns stored at sigma16(j), so that the A operand
// of K-step kk is the contiguous row 4q + kk; the diagonal tiles as they are (lower part
// zeroed), followed by the n reciprocals of the diagonal.  Used when the tiles fit
// (n <= 128); wider T is read from global memory.
template <int JT, bool kLdsT>
__global__ __launch_bounds__(256, 2) void k_trsm_ru_f64(int64_t m, int n,
                                                        const double* __restrict__ Y,
                                                        int64_t ldy,
                                                        const double* __restrict__ T,
                                                        int64_t ldt, double* X, int64_t ldx) {
  constexpr int NT = JT * (JT + 1) / 2;
  constexpr int DINV = kLdsT ? NT * 256 : 0;  // offset of the reciprocals in LDS
  extern __shared__ double tl[];
  auto Tglob = [&](const double* Tp, int i, int j) -> double {
    return (i < n && j < n) ? Tp[(int64_t)j * ldt + i] : (i == j ? 1.0 : 0.0);
  };
  for (int j = threadIdx.x; j < JT * 16; j += blockDim.x) tl[DINV + j] = 1.0 / Tglob(T, j, j);
  if (kLdsT) {
    for (int e = threadIdx.x; e < NT * 256; e += blockDim.x) {
      const int t = e / 256, w = e % 256;
      const int a = tri_a(t), b = tri_b(t);
      const int i = w / 16, j = w % 16;
      if (a == b) {
        tl[e] = (i > j) ? 0.0 : Tglob(T, 16 * a + i, 16 * b + j);
      } else {
        tl[t * 256 + i * 16 + sigma16(j)] = -Tglob(T, 16 * a + i, 16 * b + j);
      }
    }
  }
  __syncthreads();

  const int lane = lane_id();
  const int q = lane >> 4, c16 = lane & 15;
  const int sc = sigma16(c16);
  const int64_t ntiles = (m + 15) / 16;
  const int64_t wstride = (int64_t)gridDim.x * (blockDim.x / kWave);
  for (int64_t tile = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id(); tile < ntiles;
       tile += wstride) {
    // Opaque per-iteration copies of the T pointers: T is loop invariant, and without them
    // the compiler hoists every T value of every block out of the tile loop and spills.
    const double* Tp = T;
    lds_f64* tlp = (lds_f64*)tl;
    asm volatile("" : "+s"(Tp), "+v"(tlp));
    // diagonal-tile entry T(16b + i, 16b + j), i <= j
    auto Td = [&](int b, int i, int j) -> double {
      return kLdsT ? tlp[tri_index(b, b) * 256 + i * 16 + j] : Tglob(Tp, 16 * b + i, 16 * b + j);
    };
    // A operand of K-step kk for the update of block bb by block b: -T(16b+4q+kk, 16bb+sc)
    auto Aop = [&](int b, int bb, int kk) -> double {
      return kLdsT ? tlp[tri_index(b, bb) * 256 + (4 * q + kk) * 16 + c16]
                   : -Tglob(Tp, 16 * b + 4 * q + kk, 16 * bb + sc);
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
      // --- substitution on the diagonal block b, one column quad at a time
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int cb = 4 * qq;
        if (q == qq) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double x = xr[b][r] * tlp[DINV + 16 * b + cb + r];
            xr[b][r] = x;
#pragma unroll
            for (int r2 = r + 1; r2 < 4; ++r2) xr[b][r2] -= x * Td(b, cb + r, cb + r2);
          }
        }
        if (qq < 3) {
          double y[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) y[r] = __shfl(xr[b][r], c16 + 16 * qq, kWave);
          if (q > qq) {
#pragma unroll
            for (int r2 = 0; r2 < 4; ++r2) {
              double acc = xr[b][r2];
#pragma unroll
              for (int r = 0; r < 4; ++r) acc -= y[r] * Td(b, cb + r, 4 * q + r2);
              xr[b][r2] = acc;
            }
          }
        }
      }
      // --- right-looking update of the later blocks on the matrix cores
#pragma unroll
      for (int bb = b + 1; bb < JT; ++bb) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) xr[bb] = mfma_f64(Aop(b, bb, kk), xr[b][kk], xr[bb]);
      }
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

hipError_t launch_trsm(int64_t m, int n, const double* Y, int64_t ldy, const double* T,
                       int64_t ldt, double* X, int64_t ldx, hipStream_t st) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const int jt = (n + 15) / 16;
  const int64_t ntiles = (m + 15) / 16;
  int64_t blocks = (ntiles + 3) / 4;
  const int64_t cap = (int64_t)device_cu_count() * 8;
  if (blocks > cap) blocks = cap;
  dim3 grid((unsigned)blocks), block(256);
#define TSQR_TRSM(J, L)                                                                     \
  if (jt <= J) {                                                                            \
    const size_t sh = ((L ? (size_t)J * (J + 1) / 2 * 256 : 0) + 16 * J) * sizeof(double);  \
    hipLaunchKernelGGL((k_trsm_ru_f64<J, L>), grid, block, sh, st, m, n, Y, ldy, T, ldt, X, \
                       ldx);                                                                \
    return hipGetLastError();                                                               \
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

// W(i, j) = W(j, i) = sum_kb part[kb][tile][lane][reg] in fixed kb order.
__global__ void k_gram_reduce(int kblocks, int ntiles, int n, const double* __restrict__ part,
                              double* __restrict__ W, int64_t ldw) {
  const size_t E = (size_t)ntiles * 256;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < E;
       e += (size_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int kb = 0; kb < kblocks; ++kb) acc += part[(size_t)kb * E + e];
    const int tile = (int)(e / 256), lane = (int)((e / 4) % 64), r = (int)(e % 4);
    const int a = tri_a(tile), b = tri_b(tile);
    const int i = 16 * a + 4 * r + (lane >> 4), j = 16 * b + (lane & 15);
    if (i < n && j < n) {
      W[(int64_t)j * ldw + i] = acc;
      W[(int64_t)i * ldw + j] = acc;
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
  int blocks = (int)((E + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_gram_reduce, dim3(blocks), dim3(256), 0, st, p.kblocks, p.ntiles, n, part,
                     W, ldw);
  return hipGetLastError();
}

}  // namespace tsqr
