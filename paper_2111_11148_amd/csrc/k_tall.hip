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

// Prepared operand buffer, tiles of 256 doubles stored as tile[i*16 + sigma16(j)]:
//   [0, NOFF)          off-diagonal tiles (a < b): -T(16a+i, 16b+j)
//   [NOFF, NOFF+JT)    diagonal tiles: -T(16b+i, 16b+j) for i <= j, else 0
//   [NOFF+JT, +2JT)    inverted diagonal tiles: (T_bb^{-1})(i, j)
// then JT ints: 1 if the block needs the correction step.
constexpr double kTrsmRefineCond = 16.0;

__host__ __device__ constexpr size_t trsm_prep_doubles(int jt) {
  return (size_t)(jt * (jt - 1) / 2 + 2 * jt) * 256 + (size_t)(jt + 1) / 2 + 1;
}

__device__ __forceinline__ void trsm_prep_body(int n, int jt, const double* __restrict__ T,
                                               int64_t ldt, double* __restrict__ P, int b) {
  // b: block column handled by this workgroup
  const int noff = jt * (jt - 1) / 2;
  auto Tg = [&](int i, int j) -> double {
    return (i < n && j < n) ? T[(int64_t)j * ldt + i] : (i == j ? 1.0 : 0.0);
  };
  // off-diagonal tiles of block column b: one element per thread per tile, eight tiles'
  // loads in flight together
  for (int a0 = 0; a0 < b; a0 += 8)
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
      const int i = e / 16, j = e % 16;
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = (a0 + u < b) ? Tg(16 * (a0 + u) + i, 16 * b + j) : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (a0 + u < b) P[(size_t)off_index(a0 + u, b) * 256 + i * 16 + sigma16(j)] = -v[u];
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
  if (threadIdx.x < 16) {  // column j of the inverse by back substitution, in registers
    // (x[k] = 0 for k > j, so the terms past j add exact zeros after the same sum)
    const int j = threadIdx.x;
    double x[16];
#pragma unroll
    for (int i = 15; i >= 0; --i) {
      double acc = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int k = i + 1; k < 16; ++k) acc -= tb[i][k] * x[k];
      x[i] = (i <= j) ? acc / tb[i][i] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) ti[i][j] = x[i];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 256; e += blockDim.x) {
    const int i = e / 16, j = e % 16;
    P[(size_t)(noff + jt + b) * 256 + i * 16 + sigma16(j)] = ti[i][j];
  }
  if (threadIdx.x < 64) {  // infinity-norm condition estimate of the block, one wavefront
    // lane i < 16 sums row i of the block and of its inverse; the maxima over the rows by
    // DPP within the first row of 16 lanes (max is order-independent)
    const int i = threadIdx.x;
    double st = 0.0, si = 0.0;
    if (i < 16)
      for (int j = 0; j < 16; ++j) {
        st += fabs(tb[i][j]);
        si += fabs(ti[i][j]);
      }
    st = fmax(st, dpp_f64<0xB1>(st));
    st = fmax(st, dpp_f64<0x4E>(st));
    st = fmax(st, dpp_f64<0x124>(st));
    st = fmax(st, dpp_f64<0x128>(st));
    si = fmax(si, dpp_f64<0xB1>(si));
    si = fmax(si, dpp_f64<0x4E>(si));
    si = fmax(si, dpp_f64<0x124>(si));
    si = fmax(si, dpp_f64<0x128>(si));
    if (i == 0) {
      const double c = st * si;
      int* flags = reinterpret_cast<int*>(P + (size_t)(noff + 2 * jt) * 256);
      flags[b] = (c > kTrsmRefineCond || !(c == c)) ? 1 : 0;
    }
  }
}

__global__ __launch_bounds__(256) void k_trsm_prep(int n, int jt, const double* __restrict__ T,
                                                   int64_t ldt, double* __restrict__ P,
                                                   const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  trsm_prep_body(n, jt, T, ldt, P, (int)blockIdx.x);
}

typedef __attribute__((address_space(3))) int lds_int;

// The substitution of one 16-row tile held in registers (layout above): xr holds C = Y on
// entry and X on exit.  Aop(t, kk) is the A operand of prepared tile t at K-step kk;
// flags[b] selects the correction step of diagonal block b.
template <int JT, class AopF>
__device__ __forceinline__ void trsm_tile_solve(v4d (&xr)[JT], AopF Aop, const lds_int* flags) {
  constexpr int NOFF = JT * (JT - 1) / 2;
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
}

// TRSM launch shape: 16 wavefronts per workgroup, each tile loaded at the start of its own
// iteration (measured: loading the next tile one iteration ahead, with 8 wavefronts for
// the registers it needs, is not faster)
constexpr int kTrsmThreads = 1024;
// Body of workgroup `wg` of `nwg` (persistent over 16-row tiles).
template <int JT, bool kLds>
__device__ __forceinline__ void trsm_mfma_body(int64_t m, int n, const double* __restrict__ Y,
                                               int64_t ldy, const double* __restrict__ P,
                                               double* X, int64_t ldx, int wg, int nwg) {
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
  const int64_t wstride = (int64_t)nwg * nw;
  typedef __attribute__((address_space(1))) const double g_f64;
  // Y(row, 16b + 4q + r) of a tile into x[b][r]; a row past m reads row 0 and a column
  // past n reads column 0 of the same row (valid addresses: column 4q itself need not
  // exist when n <= 12), both replaced by zero
  auto load_tile = [&](int64_t tile, v4d (&x)[JT]) {
    const int64_t row = tile * 16 + c16;
    const bool rok = row < m;
    g_f64* yb = (g_f64*)(Y + (rok ? row : 0) + (int64_t)(4 * q) * ldy);
    int lim = n - 4 * q;  // column 16b + 4q + r exists iff 16b + r < lim
    int64_t cstep = uniform_i64(ldy);
    asm volatile("" : "+v"(yb), "+v"(lim), "+s"(cstep));
    const int64_t back = -(int64_t)(4 * q) * cstep;  // from column 4q back to column 0
#pragma unroll
    for (int b = 0; b < JT; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool ok = 16 * b + r < lim;
        const double v = yb[ok ? (16 * b + r) * cstep : back];
        x[b][r] = (rok && ok) ? v : 0.0;
      }
  };

  int64_t tile = (int64_t)wg * nw + wave_id();
  v4d xr[JT];
  for (; tile < ntiles; tile += wstride) {
    load_tile(tile, xr);
    // opaque per-iteration bases: the tiles are loop invariant and would otherwise be
    // hoisted into registers
    lds_f64* tlp = (lds_f64*)tl;
    const double* Pg = uniform_ptr(P);
    asm volatile("" : "+v"(tlp), "+s"(Pg));
    auto Aop = [&](int t, int kk) -> double {
      const int o = t * 256 + (4 * q + kk) * 16 + c16;
      return kLds ? tlp[o] : Pg[o];
    };
    const int64_t row = tile * 16 + c16;
    const bool rok = row < m;
    // raised issue priority during the solve, so that the arbiter prefers this wave's MFMA
    // chain over other waves' loads and stores (measured: 2^20 x 128, 0.494 -> 0.482 ms)
    __builtin_amdgcn_s_setprio(1);

    trsm_tile_solve<JT>(xr, Aop, (const lds_int*)flags);
    __builtin_amdgcn_s_setprio(0);
    if (rok) {
      // opaque base and uniform column offsets (per-lane column products would be hoisted)
      double* xb = X + row + (int64_t)(4 * q) * ldx;
      int64_t xs = uniform_i64(ldx);
      asm volatile("" : "+v"(xb), "+s"(xs));
#pragma unroll
      for (int b = 0; b < JT; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (16 * b + 4 * q + r < n) xb[(16 * b + r) * xs] = xr[b][r];
    }
  }
}

template <int JT, bool kLds>
__global__ __launch_bounds__(kTrsmThreads, 1) void k_trsm_mfma(int64_t m, int n,
                                                      const double* __restrict__ Y, int64_t ldy,
                                                      const double* __restrict__ P,
                                                      double* X, int64_t ldx,
                                                      const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  trsm_mfma_body<JT, kLds>(m, n, Y, ldy, P, X, ldx, (int)blockIdx.x, (int)gridDim.x);
}

constexpr int kBlk = 128;  // column block of the blocked solve

// A later column block of the blocked solve in one pass: C = Y - X0 T(0:K, block) against
// all solved blocks, then the block's own substitution, without writing C.  Persistent
// workgroups of 16 wavefronts take 256 rows per round (one 16-row tile per wavefront);
// the block's prepared diagonal tiles (k_trsm_prep) sit in LDS for the whole launch, and
// T(0:K, block) streams through LDS in 32-row chunks with its columns in sigma16 order,
// so that the update's accumulators come out in the substitution's register layout
// (lane (q, c16), register r of tile b = column 16b + 4q + r of row c16).  Y may be the
// output block itself (each element is read and written by the same lane).
template <int JT>
__global__ __launch_bounds__(1024, 1) void k_trsm_fused(int64_t m, int n, int K,
                                                       const double* __restrict__ X0,
                                                       int64_t ldx0,
                                                       const double* __restrict__ Tk,
                                                       int64_t ldt, const double* Y, int64_t ldy,
                                                       const double* __restrict__ P, double* Xk,
                                                       int64_t ldxk,
                                                       const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  constexpr int NOFF = JT * (JT - 1) / 2;
  constexpr int NTILE = NOFF + 2 * JT;
  constexpr int KCH = 32;          // rows of T per staged chunk (8 K-steps)
  constexpr int NC = 16 * JT;      // columns of the block (padded)
  constexpr int LDU = NC + 1;
  extern __shared__ double sm[];
  double* tl = sm;                 // prepared diagonal tiles
  double* tu = sm + NTILE * 256;   // KCH x LDU chunk of T(0:K, block)
  __shared__ int flags[JT];
  const int* flags_g = reinterpret_cast<const int*>(P + (size_t)NTILE * 256);
  for (int e = threadIdx.x; e < NTILE * 256; e += blockDim.x) tl[e] = P[e];
  for (int e = threadIdx.x; e < JT; e += blockDim.x) flags[e] = flags_g[e];

  const int lane = lane_id(), wave = wave_id();
  const int q = lane >> 4, c16 = lane & 15;
  const int64_t ntiles = (m + 15) / 16;
  const int64_t ngroups = (ntiles + 15) / 16;
  for (int64_t g = blockIdx.x; g < ngroups; g += gridDim.x) {
    const int64_t tile = g * 16 + wave;
    const int64_t row = tile * 16 + c16;
    const bool rok = tile < ntiles && row < m;
    const int64_t rowc = rok ? row : 0;  // clamped, always a valid address
    v4d xr[JT];
#pragma unroll
    for (int b = 0; b < JT; ++b) xr[b] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < K; kc += KCH) {
      // this chunk's X0(row, kc + 4j + q), issued before the barriers
      double xa[KCH / 4];
      {
        const double* xp = X0 + (int64_t)(kc + q) * ldx0 + rowc;
        int64_t xs = ldx0;
        asm volatile("" : "+v"(xp), "+s"(xs));
#pragma unroll
        for (int j = 0; j < KCH / 4; ++j) xa[j] = xp[(4 * j) * xs];
      }
      __syncthreads();  // the previous chunk (or round) is done with tu
      for (int e = threadIdx.x; e < KCH * NC; e += blockDim.x) {
        const int k = e % KCH, pcol = e / KCH;  // consecutive threads: consecutive rows
        const int col = 16 * (pcol / 16) + sigma16(pcol % 16);
        tu[k * LDU + pcol] = (col < n) ? Tk[(int64_t)col * ldt + kc + k] : 0.0;
      }
      __syncthreads();
#pragma unroll
      for (int j = 0; j < KCH / 4; ++j) {
        const lds_f64* tp = (const lds_f64*)tu + (4 * j + q) * LDU + c16;
        asm volatile("" : "+v"(tp));
        const double xv = rok ? xa[j] : 0.0;
#pragma unroll
        for (int b = 0; b < JT; ++b) xr[b] = mfma_f64(tp[16 * b], xv, xr[b]);
      }
    }
    __syncthreads();  // tl and flags are staged (first round)
    // C = Y - X0 T, in place in xr
    {
      const double* yb = Y + rowc + (int64_t)(4 * q) * ldy;
      int64_t ys = ldy;
      int lim = n - 4 * q;  // column 16b + 4q + r exists iff 16b + r < lim
      asm volatile("" : "+v"(yb), "+s"(ys), "+v"(lim));
#pragma unroll
      for (int b = 0; b < JT; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const bool ok = 16 * b + r < lim;
          const double y = yb[ok ? (16 * b + r) * ys : 0];
          xr[b][r] = (rok && ok) ? y - xr[b][r] : 0.0;
        }
    }
    // the block's substitution (as in trsm_mfma_body)
    lds_f64* tlp = (lds_f64*)tl;
    asm volatile("" : "+v"(tlp));
    auto Aop = [&](int t, int kk) -> double { return tlp[t * 256 + (4 * q + kk) * 16 + c16]; };
#pragma unroll
    for (int b = 0; b < JT; ++b) {
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
#pragma unroll
      for (int bb = b + 1; bb < JT; ++bb)
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
          xr[bb] = mfma_f64(Aop(off_index(b, bb), kk), xr[b][kk], xr[bb]);
    }
    if (rok) {
      double* xb = Xk + row + (int64_t)(4 * q) * ldxk;
      int64_t xs = ldxk;
      asm volatile("" : "+v"(xb), "+s"(xs));
#pragma unroll
      for (int b = 0; b < JT; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (16 * b + 4 * q + r < n) xb[(16 * b + r) * xs] = xr[b][r];
    }
  }
}

size_t trsm_scratch_doubles(int n) {
  // wider matrices are solved in column blocks of kBlk that reuse one prepared block
  const int nn = n > kBlk ? kBlk : n;
  int jt = 1;
  while (jt < (nn + 15) / 16) jt <<= 1;
  return trsm_prep_doubles(jt);
}

static hipError_t launch_trsm_block(int64_t m, int n, const double* Y, int64_t ldy,
                                    double* X, int64_t ldx, double* scratch, hipStream_t st,
                                    const int* gate);

// Operand preparation of the first column block (all of T up to kBlk columns).
hipError_t launch_trsm_prepare(int n, const double* T, int64_t ldt, double* scratch,
                               hipStream_t st, const int* gate) {
  if (n <= 0) return hipSuccess;
  const int nb = n < kBlk ? n : kBlk;
  int jt = 1;
  while (jt < (nb + 15) / 16) jt <<= 1;
  hipLaunchKernelGGL(k_trsm_prep, dim3(jt), dim3(256), 0, st, nb, jt, T, ldt, scratch, gate);
  return hipGetLastError();
}

// X = Y T^{-1} after launch_trsm_prepare.  Up to kBlk columns: one substitution kernel.
// Wider: by column blocks of kBlk; the first block is the substitution kernel, every later
// block one pass of k_trsm_fused (update against all solved blocks, then the block's own
// substitution).
hipError_t launch_trsm_solve(int64_t m, int n, const double* Y, int64_t ldy, const double* T,
                             int64_t ldt, double* X, int64_t ldx, double* scratch,
                             hipStream_t st, const int* gate) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (n <= kBlk) return launch_trsm_block(m, n, Y, ldy, X, ldx, scratch, st, gate);
  const int64_t ntiles = (m + 15) / 16;
  const int64_t cap = (int64_t)device_cu_count();
  hipError_t e = launch_trsm_block(m, kBlk, Y, ldy, X, ldx, scratch, st, gate);
  if (e != hipSuccess) return e;
  for (int k0 = kBlk; k0 < n; k0 += kBlk) {
    const int nbk = (n - k0) < kBlk ? (n - k0) : kBlk;
    int jt = 1;
    while (jt < (nbk + 15) / 16) jt <<= 1;
    hipLaunchKernelGGL(k_trsm_prep, dim3(jt), dim3(256), 0, st, nbk, jt,
                       T + (int64_t)k0 * ldt + k0, ldt, scratch, gate);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t ngroups = (ntiles + 15) / 16;
    const int64_t grid = ngroups < cap ? ngroups : cap;
    const double* yk = Y + (int64_t)k0 * ldy;
    double* xk = X + (int64_t)k0 * ldx;
#define TSQR_TF(J)                                                                             \
  if (jt == J) {                                                                               \
    const size_t sh = ((size_t)(J * (J - 1) / 2 + 2 * J) * 256 + 32 * (16 * J + 1)) * sizeof(double); \
    hipLaunchKernelGGL(k_trsm_fused<J>, dim3((unsigned)grid), dim3(1024), sh, st, m, nbk, k0, X,  \
                       ldx, T + (int64_t)k0 * ldt, ldt, yk, ldy, scratch, xk, ldx, gate);             \
  }
    TSQR_TF(1) TSQR_TF(2) TSQR_TF(4) TSQR_TF(8)
#undef TSQR_TF
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_trsm(int64_t m, int n, const double* Y, int64_t ldy, const double* T,
                       int64_t ldt, double* X, int64_t ldx, double* scratch, hipStream_t st,
                       const int* gate) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const hipError_t e = launch_trsm_prepare(n, T, ldt, scratch, st, gate);
  if (e != hipSuccess) return e;
  return launch_trsm_solve(m, n, Y, ldy, T, ldt, X, ldx, scratch, st, gate);
}

// The substitution kernel over up to kBlk columns, operands prepared in `scratch`.
static hipError_t launch_trsm_block(int64_t m, int n, const double* Y, int64_t ldy,
                                    double* X, int64_t ldx, double* scratch, hipStream_t st,
                                    const int* gate) {
  int jt = 1;
  while (jt < (n + 15) / 16) jt <<= 1;
  if (jt > 8) return hipErrorInvalidValue;
  const int64_t ntiles = (m + 15) / 16;
  int64_t blocks = (ntiles + kTrsmThreads / 64 - 1) / (kTrsmThreads / 64);
  const int64_t cap = (int64_t)device_cu_count();
  if (blocks > cap) blocks = cap;
  dim3 grid((unsigned)blocks), block(kTrsmThreads);
#define TSQR_TRSM(J, L)                                                                    \
  if (jt == J) {                                                                           \
    const size_t sh = L ? (size_t)(J * (J - 1) / 2 + 2 * J) * 256 * sizeof(double) : 0;    \
    hipLaunchKernelGGL((k_trsm_mfma<J, L>), grid, block, sh, st, m, n, Y, ldy, scratch, X, \
                       ldx, gate);                                                         \
    return hipGetLastError();                                                              \
  }
  TSQR_TRSM(1, true) TSQR_TRSM(2, true) TSQR_TRSM(4, true) TSQR_TRSM(8, true)
#undef TSQR_TRSM
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------------------
// Gram matrix W = X^T X (upper 16x16 tiles), split over row blocks.  A workgroup streams
// its row block in 32-row chunks: the next chunk is loaded into registers (16-byte loads,
// two rows of one column per thread) while the current one, staged row-major in LDS, feeds
// the matrix cores, so global latency hides behind the MFMA work with one barrier pair per
// chunk.  For MFMA K-step kk, lane l reads X(row 4kk + l/16, col 16c + l%16), which is
// simultaneously the A operand (X^T) of tile (c, .) and the B operand of (., c).  Wave w
// owns the upper tiles t = w, w + NW, ... (tiles numbered column by column); the tile set
// is a compile-time property of the wave (gram_chunk<..., W>), so the inner loop is a
// straight run of MFMAs with no per-tile branches.  For wide matrices the tiles are also
// shared out over NS workgroups per row block (blockIdx.y): slot y NW + w owns tiles
// slot, slot + NS NW, ...  Partials are written tile-natively and summed in a fixed order
// by k_gram_reduce.
// ------------------------------------------------------------------------------------
// One K-step of wave W: acc[u] += X(:, a)^T X(:, b) for its tiles t = W + u NW.
template <int STRIDE, int W, int TPW, int... U>
__device__ __forceinline__ void gram_step(const double* op, v4d (&acc)[TPW],
                                          std::integer_sequence<int, U...>) {
  ((acc[U] = mfma_f64(op[UpperTile<W + U * STRIDE>::a], op[UpperTile<W + U * STRIDE>::b],
                      acc[U])),
   ...);
}

template <int JT, int STRIDE, int W, int KC, int LDN, int TPW>
__device__ __forceinline__ void gram_chunk(const lds_f64* lds, int q, int c16, v4d (&acc)[TPW]) {
  constexpr int NT = JT * (JT + 1) / 2;
  constexpr int CNT = NT > W ? (NT - W + STRIDE - 1) / STRIDE : 0;
  const lds_f64* lp = lds + q * LDN + c16;
#pragma unroll
  for (int kk = 0; kk < KC / 4; ++kk) {
    const lds_f64* rowp = lp + 4 * kk * LDN;
    double op[JT];
#pragma unroll
    for (int c = 0; c < JT; ++c) op[c] = rowp[16 * c];
    gram_step<STRIDE, W, TPW>(op, acc, std::make_integer_sequence<int, CNT>{});
  }
}

// VEC: X is 16-byte aligned, ldx and m are even, so every in-range row pair is one
// aligned 16-byte load (chosen on the host; the loads stay branch-free either way, so the
// prefetch is never waited for before the MFMA work that should hide it).
// Body of workgroup (row block bx, tile share by).  EXTL: the chunk buffers live at
// ext_lds (gram_f64_lds_doubles<JT>() doubles) instead of in the body's own LDS.
template <int JT>
__host__ __device__ constexpr int gram_f64_lds_doubles() {
  return 2 * 32 * (JT * 16 + 1);
}

template <int JT, int NW, int NS, bool VEC, bool EXTL = false>
__device__ __forceinline__ void gram_f64_body(int64_t m, int n, const double* __restrict__ X,
                                              int64_t ldx, int64_t rows_per_block, int ntiles,
                                              double* __restrict__ part, int bx, int by,
                                              double* ext_lds = nullptr) {
  constexpr int KC = 32;
  constexpr int NC = JT * 16;
  constexpr int LDN = NC + 1;
  constexpr int NT = JT * (JT + 1) / 2;
  constexpr int STRIDE = NW * NS;
  constexpr int TPW = (NT + STRIDE - 1) / STRIDE;
  constexpr int THREADS = NW * 64;
  constexpr int CPP = THREADS / (KC / 2);  // columns loaded per pass
  constexpr int PASSES = (NC + CPP - 1) / CPP;
  static_assert(STRIDE <= 16, "slot dispatch covers at most 16 slots");
  // double buffer: one barrier per chunk
  double* lbase;
  if constexpr (EXTL) {
    lbase = ext_lds;
  } else {
    __shared__ double own[2 * KC * LDN];
    lbase = own;
  }
  double(*lds)[KC * LDN] = reinterpret_cast<double(*)[KC * LDN]>(lbase);

  const int lane = lane_id(), wave = wave_id();
  const int q = lane >> 4, c16 = lane & 15;
  const int slot = by * NW + wave;
  const int64_t r0 = (int64_t)bx * rows_per_block;
  const int64_t r1 = min(m, r0 + rows_per_block);

  v4d acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) acc[u] = v4d{0.0, 0.0, 0.0, 0.0};

  // rows start even (row blocks and chunks are multiples of 32): with m even, row < r1
  // implies row + 1 < r1, and the pair (2rp, 2rp+1) is one aligned 16-byte word
  const int rp = (int)threadIdx.x % (KC / 2), cb = (int)threadIdx.x / (KC / 2);
  double pre[PASSES][2];
  auto load_chunk = [&](int64_t rb) {
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
      const int cc = cb + ps * CPP;
      const int64_t row = rb + 2 * rp;
      const bool okc = (cc < NC) && (cc < n);
      if constexpr (VEC) {
        const bool ok = okc && row < r1;
        const double* src = ok ? X + (int64_t)cc * ldx + row : X;  // clamped, always valid
        const v2d v = *reinterpret_cast<const v2d*>(src);
        pre[ps][0] = ok ? v[0] : 0.0;
        pre[ps][1] = ok ? v[1] : 0.0;
      } else {
        const double* src = X + (int64_t)cc * ldx + row;
        pre[ps][0] = (okc && row < r1) ? src[0] : 0.0;
        pre[ps][1] = (okc && row + 1 < r1) ? src[1] : 0.0;
      }
    }
  };

  auto stage = [&](double* buf) {
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
      const int cc = cb + ps * CPP;
      if (cc < NC) {
        buf[(2 * rp) * LDN + cc] = pre[ps][0];
        buf[(2 * rp + 1) * LDN + cc] = pre[ps][1];
      }
    }
  };
  // chunk c is staged in buffer c % 2 at the end of chunk c - 1's products (every wave has
  // passed the barrier after chunk c - 2, the buffer's previous user), and chunk c + 2's
  // loads are issued once chunk c + 1 is staged
  if (r0 < r1) {
    load_chunk(r0);
    stage(lds[0]);
    if (r0 + KC < r1) load_chunk(r0 + KC);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t rb = r0; rb < r1; rb += KC, cur ^= 1) {
    const lds_f64* lp = (const lds_f64*)lds[cur];
    switch (slot) {
#define TSQR_GRAM_SLOT(W_)                                                             \
  case W_:                                                                             \
    if constexpr (W_ < STRIDE) gram_chunk<JT, STRIDE, W_, KC, LDN, TPW>(lp, q, c16, acc); \
    break;
      TSQR_GRAM_SLOT(0) TSQR_GRAM_SLOT(1) TSQR_GRAM_SLOT(2) TSQR_GRAM_SLOT(3)
      TSQR_GRAM_SLOT(4) TSQR_GRAM_SLOT(5) TSQR_GRAM_SLOT(6) TSQR_GRAM_SLOT(7)
      TSQR_GRAM_SLOT(8) TSQR_GRAM_SLOT(9) TSQR_GRAM_SLOT(10) TSQR_GRAM_SLOT(11)
      TSQR_GRAM_SLOT(12) TSQR_GRAM_SLOT(13) TSQR_GRAM_SLOT(14) TSQR_GRAM_SLOT(15)
#undef TSQR_GRAM_SLOT
      default: break;
    }
    if (rb + KC < r1) stage(lds[cur ^ 1]);
    __syncthreads();
    if (rb + 2 * KC < r1) load_chunk(rb + 2 * KC);
  }

  // tiles are enumerated column by column, so the first `ntiles` are those of the
  // n x n matrix (the rest only exist in the padded template size)
  double* dst = part + (size_t)bx * ntiles * 256;
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int t = slot + u * STRIDE;
    if (t < NT && t < ntiles) *reinterpret_cast<v4d*>(dst + (size_t)t * 256 + lane * 4) = acc[u];
  }
}

template <int JT, int NW, int NS, bool VEC>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(2))) void k_gram_f64(
    int64_t m, int n, const double* __restrict__ X, int64_t ldx, int64_t rows_per_block,
    int ntiles, double* __restrict__ part,
    const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  gram_f64_body<JT, NW, NS, VEC>(m, n, X, ldx, rows_per_block, ntiles, part, (int)blockIdx.x,
                                 (int)blockIdx.y);
}

// W(i, j) = W(j, i) = sum_kb part[kb][tile][lane][reg]; same deterministic two-level
// order as the sketch reduction (16 strided groups, then the groups in order).
__device__ __forceinline__ void gram_reduce_body(int kblocks, int ntiles, int n,
                                                 const double* __restrict__ part,
                                                 double* __restrict__ W, int64_t ldw, int bx) {
  __shared__ double red[16][17];
  const size_t E = (size_t)ntiles * 256;
  const int g = threadIdx.x / 16, o = threadIdx.x % 16;
  const size_t e = (size_t)bx * 16 + o;
  double acc = 0.0;
  if (e < E) acc = strided_sum(part, E, e, g, 16, kblocks);
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

__global__ __launch_bounds__(256) void k_gram_reduce(int kblocks, int ntiles, int n,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ W, int64_t ldw,
                                                     const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  gram_reduce_body(kblocks, ntiles, n, part, W, ldw, (int)blockIdx.x);
}

// ------------------------------------------------------------------------------------
// Wide Gram matrix (n > 256): W is cut into 128 x 128 blocks.  Workgroup (row block bx,
// block pair by = (bi <= bj)) accumulates X(:, block bi)^T X(:, block bj) over its rows;
// its eight wavefronts own the eight 16-row strips of the block pair (wave a: tiles (a, b)
// for b = 0..7).  Rows are streamed in 32-row chunks through LDS with register prefetch as
// in k_gram_f64; partials are written tile-natively per (row block, pair, tile) and summed
// in a fixed order by k_gram_wide_reduce.
// ------------------------------------------------------------------------------------
constexpr int kWideBlk = 128;

__host__ __device__ inline void wide_pair(int t, int& bi, int& bj) {
  int b = 0;
  while ((b + 1) * (b + 2) / 2 <= t) ++b;
  bj = b;
  bi = t - b * (b + 1) / 2;
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_gram_wide(
    int64_t m, int n, const double* __restrict__ X, int64_t ldx, int64_t rows_per_block,
    int npairs, double* __restrict__ part,
    const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  constexpr int KC = 32, NC = kWideBlk, LDN = NC + 1;
  constexpr int THREADS = 512;
  constexpr int CPP = THREADS / (KC / 2);      // 32 columns per pass
  constexpr int PASSES = 2 * NC / CPP;         // both blocks: 8 passes
  __shared__ double la[KC * LDN];
  __shared__ double lb[KC * LDN];
  const int lane = lane_id(), wave = wave_id();
  const int q = lane >> 4, c16 = lane & 15;
  int bi, bj;
  wide_pair((int)blockIdx.y, bi, bj);
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(m, r0 + rows_per_block);
  v4d acc[8];
#pragma unroll
  for (int b = 0; b < 8; ++b) acc[b] = v4d{0.0, 0.0, 0.0, 0.0};
  const int rp = (int)threadIdx.x % (KC / 2), cb = (int)threadIdx.x / (KC / 2);
  double pre[PASSES][2];
  auto load_chunk = [&](int64_t rb) {
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
      const int cc = cb + ps * CPP;  // 0..255: first block bi, then block bj
      const int col = (cc < NC) ? kWideBlk * bi + cc : kWideBlk * bj + (cc - NC);
      const int64_t row = rb + 2 * rp;
      const bool okc = col < n;
      const double* src = X + (int64_t)(okc ? col : 0) * ldx;
      pre[ps][0] = (okc && row < r1) ? src[row] : 0.0;
      pre[ps][1] = (okc && row + 1 < r1) ? src[row + 1] : 0.0;
    }
  };
  if (r0 < r1) load_chunk(r0);
  for (int64_t rb = r0; rb < r1; rb += KC) {
    __syncthreads();
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
      const int cc = cb + ps * CPP;
      double* dst = (cc < NC) ? la + cc : lb + (cc - NC);
      dst[(2 * rp) * LDN] = pre[ps][0];
      dst[(2 * rp + 1) * LDN] = pre[ps][1];
    }
    __syncthreads();
    if (rb + KC < r1) load_chunk(rb + KC);
    const lds_f64* pa = (const lds_f64*)la + q * LDN + 16 * wave + c16;
    const lds_f64* pb = (const lds_f64*)lb + q * LDN + c16;
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const double a = pa[4 * kk * LDN];
#pragma unroll
      for (int b = 0; b < 8; ++b) acc[b] = mfma_f64(a, pb[4 * kk * LDN + 16 * b], acc[b]);
    }
  }
  double* dst = part + ((size_t)blockIdx.x * npairs + blockIdx.y) * 64 * 256;
#pragma unroll
  for (int b = 0; b < 8; ++b)
    *reinterpret_cast<v4d*>(dst + (size_t)(wave * 8 + b) * 256 + lane * 4) = acc[b];
}

// W(i, j) = W(j, i) = sum_kb part[kb][pair][tile][lane][reg], fixed two-level order; in a
// diagonal block pair only the entries with i <= j are taken (each written once).
__global__ __launch_bounds__(256) void k_gram_wide_reduce(int kblocks, int npairs, int n,
                                                          const double* __restrict__ part,
                                                          double* __restrict__ W, int64_t ldw,
                                                          const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  __shared__ double red[16][17];
  const size_t E = (size_t)npairs * 64 * 256;
  const int g = threadIdx.x / 16, o = threadIdx.x % 16;
  const size_t e = (size_t)blockIdx.x * 16 + o;
  double acc = 0.0;
  if (e < E) acc = strided_sum(part, E, e, g, 16, kblocks);
  red[g][o] = acc;
  __syncthreads();
  if (g == 0 && e < E) {
    double t = 0.0;
    for (int k = 0; k < 16; ++k) t += red[k][o];
    const int pair = (int)(e / (64 * 256)), tile = (int)((e / 256) % 64);
    const int lane = (int)((e / 4) % 64), r = (int)(e % 4);
    int bi, bj;
    wide_pair(pair, bi, bj);
    const int i = kWideBlk * bi + 16 * (tile / 8) + 4 * r + (lane >> 4);
    const int j = kWideBlk * bj + 16 * (tile % 8) + (lane & 15);
    if (i < n && j < n && (bi != bj || i <= j)) {
      W[(int64_t)j * ldw + i] = t;
      W[(int64_t)i * ldw + j] = t;
    }
  }
}

GramPlan plan_gram(int64_t m, int n) {
  GramPlan p{};
  p.jt_total = (n + 15) / 16;
  p.ntiles = p.jt_total * (p.jt_total + 1) / 2;
  if (n > 256) {
    const int nb = (n + kWideBlk - 1) / kWideBlk;
    p.wide = 1;
    p.npairs = nb * (nb + 1) / 2;
    int64_t kb = (int64_t)device_cu_count() * 2 / p.npairs;
    if (kb < 1) kb = 1;
    int64_t rpb = (m + kb - 1) / kb;
    rpb = ((rpb + 63) / 64) * 64;
    if (rpb < 64) rpb = 64;
    p.rows_per_block = rpb;
    p.kblocks = (int)((m + rpb - 1) / rpb);
    p.part_doubles = (size_t)p.kblocks * p.npairs * 64 * 256;
    return p;
  }
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
                       double* part, hipStream_t st, const int* gate) {
  if (p.wide) {
    hipLaunchKernelGGL(k_gram_wide, dim3(p.kblocks, p.npairs), dim3(512), 0, st, m, n, X, ldx,
                       p.rows_per_block, p.npairs, part, gate);
    return hipGetLastError();
  }
  const bool vec = ((reinterpret_cast<uintptr_t>(X) & 15) == 0) && ((ldx & 1) == 0) &&
                   ((m & 1) == 0);
#define TSQR_GRAM(J, NW_, NS_)                                                              \
  if (p.jt_total <= J) {                                                                   \
    const dim3 grid(p.kblocks, NS_);                                                       \
    if (vec)                                                                               \
      hipLaunchKernelGGL((k_gram_f64<J, NW_, NS_, true>), grid, dim3(NW_ * 64), 0, st, m, n, \
                         X, ldx, p.rows_per_block, p.ntiles, part, gate);                  \
    else                                                                                   \
      hipLaunchKernelGGL((k_gram_f64<J, NW_, NS_, false>), grid, dim3(NW_ * 64), 0, st, m,  \
                         n, X, ldx, p.rows_per_block, p.ntiles, part, gate);               \
    return hipGetLastError();                                                               \
  }
  TSQR_GRAM(1, 4, 1) TSQR_GRAM(2, 4, 1) TSQR_GRAM(4, 4, 1) TSQR_GRAM(8, 4, 1)
  TSQR_GRAM(16, 8, 2)
#undef TSQR_GRAM
  return hipErrorInvalidValue;
}

hipError_t launch_gram_reduce(const GramPlan& p, int n, const double* part, double* W,
                              int64_t ldw, hipStream_t st, const int* gate) {
  if (p.wide) {
    const size_t E = (size_t)p.npairs * 64 * 256;
    hipLaunchKernelGGL(k_gram_wide_reduce, dim3((unsigned)((E + 15) / 16)), dim3(256), 0, st,
                       p.kblocks, p.npairs, n, part, W, ldw, gate);
    return hipGetLastError();
  }
  const size_t E = (size_t)p.ntiles * 256;
  const int blocks = (int)((E + 15) / 16);
  hipLaunchKernelGGL(k_gram_reduce, dim3(blocks), dim3(256), 0, st, p.kblocks, p.ntiles, n, part,
                     W, ldw, gate);
  return hipGetLastError();
}

// ---- batched forms ----------------------------------------------------------------------
__device__ __forceinline__ const double* b_factor(const BProb& p, int which) {
  return which == 0 ? p.R0 : (which == 1 ? p.R1 : p.R2);
}

__global__ __launch_bounds__(256) void k_b_trsm_prep(int which, const BItem* __restrict__ items,
                                                     const BProb* __restrict__ probs) {
  const BItem it = items[blockIdx.x];
  const BProb& p = probs[it.pid];
  int jt = 1;
  while (jt < (p.n + 15) / 16) jt <<= 1;
  trsm_prep_body(p.n, jt, b_factor(p, which), p.n, p.P, it.x);
}

template <int JT>
__global__ __launch_bounds__(512, 1) void k_b_trsm(int src, const BItem* __restrict__ items,
                                                   const BProb* __restrict__ probs) {
  const BItem it = items[blockIdx.x];
  const BProb& p = probs[it.pid];
  const double* Y = src == 0 ? p.A : p.Q;
  const int64_t ldy = src == 0 ? p.lda : p.ldq;
  trsm_mfma_body<JT, true>(p.m, p.n, Y, ldy, p.P, p.Q, p.ldq, it.x, p.trsm_wgs);
}

template <int JT, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(2))) void k_b_gram(
    const BItem* __restrict__ items, const BProb* __restrict__ probs) {
  const BItem it = items[blockIdx.x];
  const BProb& p = probs[it.pid];
  gram_f64_body<JT, NW, 1, false>(p.m, p.n, p.Q, p.ldq, p.gr_rpb, p.gr_ntiles, p.part, it.x, 0);
}

__global__ __launch_bounds__(256) void k_b_gram_reduce(const BItem* __restrict__ items,
                                                       const BProb* __restrict__ probs) {
  const BItem it = items[blockIdx.x];
  const BProb& p = probs[it.pid];
  gram_reduce_body(p.gr_kblocks, p.gr_ntiles, p.n, p.part, p.W, p.n, it.x);
}

hipError_t launch_b_trsm_prep(int which, const BItem* items, int nitems, const BProb* probs,
                              hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_trsm_prep, dim3(nitems), dim3(256), 0, st, which, items, probs);
  return hipGetLastError();
}

hipError_t launch_b_trsm(int JT, int src, const BItem* items, int nitems, const BProb* probs,
                         hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
#define TSQR_BTR(J)                                                                           \
  if (JT == J) {                                                                              \
    const size_t sh = (size_t)(J * (J - 1) / 2 + 2 * J) * 256 * sizeof(double);               \
    hipLaunchKernelGGL((k_b_trsm<J>), dim3(nitems), dim3(512), sh, st, src, items, probs);    \
    return hipGetLastError();                                                                 \
  }
  TSQR_BTR(1) TSQR_BTR(2) TSQR_BTR(4) TSQR_BTR(8)
#undef TSQR_BTR
  return hipErrorInvalidValue;
}

hipError_t launch_b_gram(int JT, const BItem* items, int nitems, const BProb* probs,
                         hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
#define TSQR_BGR(J)                                                                           \
  if (JT == J) {                                                                              \
    hipLaunchKernelGGL((k_b_gram<J, 4>), dim3(nitems), dim3(256), 0, st, items, probs);       \
    return hipGetLastError();                                                                 \
  }
  TSQR_BGR(1) TSQR_BGR(2) TSQR_BGR(4) TSQR_BGR(8)
#undef TSQR_BGR
  return hipErrorInvalidValue;
}

hipError_t launch_b_gram_reduce(const BItem* items, int nitems, const BProb* probs,
                                hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_gram_reduce, dim3(nitems), dim3(256), 0, st, items, probs);
  return hipGetLastError();
}

}  // namespace tsqr
