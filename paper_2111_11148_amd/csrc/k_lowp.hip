// Low-precision phases of the mixed-precision variant: the sketch B = S A, the
// preconditioner apply A1 = A R0^{-1} (with the explicit inverse, computed in FP64 and
// rounded) and the first Gram matrix A1^T A1, each with FP32 or BF16 inputs on the
// matrix cores and FP32 accumulation; partial sums are kept in FP64.
//
// MFMA shapes (gfx950): V_MFMA_F32_16X16X4_F32 (one FP32 value per lane and operand, K = 4)
// and V_MFMA_F32_16X16X32_BF16 (eight BF16 values per lane, K = 32).  In both, lane l
// supplies A[l%16][KPL*(l/16) + e] and B[KPL*(l/16) + e][l%16] (e < KPL) and holds
// D[4*(l/16) + r][l%16] in register r.
//
// Roundings: FP64 -> FP32 is round-to-nearest-even; BF16 is the round-to-nearest-even
// BF16 of that FP32 value (two roundings, kept apart on purpose: see LowT).  Sketch normals
// are FP32 numbers (BF16 path: rounded to BF16).  The sketch takes A as its FP32 rounding
// for both input types: on the BF16 path that value is staged as three BF16 numbers whose
// sum is exactly it (LowT<BF16>::split3), and each step issues three BF16 MFMAs on the same
// normals, whose products are exact in the FP32 accumulator.
#include "tsqr_device.hpp"
#include "tsqr_launch.hpp"

namespace tsqr {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

__device__ __forceinline__ v4f mfma_f32(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4f mfma_bf16(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int PREC>
struct LowT;
template <>
struct LowT<TSQR_LOWP_FP32> {
  typedef float E;
  static __device__ __forceinline__ E from_double(double x) { return (float)x; }
  static __device__ __forceinline__ E from_float(float x) { return x; }
};
template <>
struct LowT<TSQR_LOWP_BF16> {
  typedef __bf16 E;
  // Two roundings, FP64 -> FP32 -> BF16, each to nearest even.  The compiler would
  // otherwise fuse the pair into one correctly rounded FP64 -> BF16 conversion (a
  // different value for inputs near a BF16 midpoint, and a longer instruction sequence);
  // the empty asm makes the FP32 value opaque so both roundings happen as written.
  static __device__ __forceinline__ E from_double(double x) {
    float f = (float)x;
    asm volatile("" : "+v"(f));
    return (__bf16)f;
  }
  static __device__ __forceinline__ E from_float(float x) { return (__bf16)x; }
  // x rounded to FP32, then written as hi + mid + lo exactly: hi is the BF16 rounding of
  // that FP32 value, mid the BF16 rounding of the remainder, lo the remainder after that.
  // Each remainder is an exact FP32 difference (a number minus its own rounding to fewer
  // bits), and the last one has at most 8 significant bits, so lo is exact too.
  static __device__ __forceinline__ void split3(double x, E& hi, E& mid, E& lo) {
    float f = (float)x;
    asm volatile("" : "+v"(f));
    hi = (__bf16)f;
    const float r1 = f - (float)hi;
    mid = (__bf16)r1;
    const float r2 = r1 - (float)mid;
    lo = (__bf16)r2;
  }
};

// value D[i][j] held at (lane, reg) in the low-precision accumulator layout goes to the
// FP64 tile-native position (16*reg + lane%16, lane/16) used by the partial-sum reductions
__device__ __forceinline__ int lowp_to_f64_tile_index(int lane, int r) {
  return (16 * r + (lane & 15)) * 4 + (lane >> 4);
}

// ===================================================================== sketch ====
// One workgroup: a row block of A, i-tiles it0.. of B for each wavefront, JT column tiles.
// A is staged in LDS column-major (rows contiguous) already rounded to the input type.
// Body of workgroup (row block bx, i-group by, column group bz).  EXTL: the staging buffer
// lives at ext_lds (sketch_lowp_lds_bytes<PREC, JT>() bytes, 16-byte aligned) instead of in
// the body's own LDS.
// (BF16: three planes, the hi, mid and lo terms of A)
template <int PREC, int JT>
__host__ __device__ constexpr int sketch_lowp_lds_bytes() {
  return JT * 16 * ((PREC == TSQR_LOWP_FP32) ? 65 : 72) * ((PREC == TSQR_LOWP_FP32) ? 4 : 6);
}

template <int PREC, int IT, int JT, int NW, bool EXTL = false>
__device__ __forceinline__ void sketch_lowp_body(
    int64_t m, int n, const double* __restrict__ A, int64_t lda, uint32_t k0, uint32_t k1,
    int64_t rows_per_block, int it_total, int jt_total, double* __restrict__ part, int bx,
    int by, int bz, double* ext_lds = nullptr) {
  typedef typename LowT<PREC>::E E;
  constexpr int KC = 64;                       // rows per chunk
  constexpr int NC = JT * 16;
  constexpr int LDR = (PREC == TSQR_LOWP_FP32) ? KC + 1 : KC + 8;
  constexpr int T = NW * 64;
  constexpr int PLANES = (PREC == TSQR_LOWP_FP32) ? 1 : 3;
  constexpr int PL = NC * LDR;  // elements per plane
  static_assert(PLANES * PL * (int)sizeof(E) == sketch_lowp_lds_bytes<PREC, JT>(), "LDS size");
  E* lds;
  if constexpr (EXTL) {
    lds = reinterpret_cast<E*>(ext_lds);
  } else {
    __shared__ __attribute__((aligned(16))) E own[PLANES * PL];
    lds = own;
  }

  const int lane = lane_id(), wave = wave_id();
  const int q = lane >> 4, c16 = lane & 15;
  const int64_t r0 = (int64_t)bx * rows_per_block;
  const int64_t r1 = min(m, r0 + rows_per_block);
  const int it0 = by * (NW * IT) + wave * IT;
  const int c0 = bz * NC;

  v4f acc[IT][JT];
  v4d acc64[IT][JT];
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) {
      acc[it][jt] = v4f{0.f, 0.f, 0.f, 0.f};
      acc64[it][jt] = v4d{0.0, 0.0, 0.0, 0.0};
    }

  for (int64_t rb = r0; rb < r1; rb += KC) {
    __syncthreads();
    if constexpr (PREC == TSQR_LOWP_FP32) {
      for (int e = threadIdx.x; e < KC * NC; e += T) {
        const int rr = e % KC, cc = e / KC;
        const int64_t row = rb + rr;
        const int col = c0 + cc;
        const double v = (row < r1 && col < n) ? A[(int64_t)col * lda + row] : 0.0;
        lds[cc * LDR + rr] = LowT<PREC>::from_double(v);
      }
    } else {
      // row pairs: one LDS write per plane for two elements (rr and LDR even)
      for (int e = threadIdx.x; e < KC / 2 * NC; e += T) {
        const int rr = 2 * (e % (KC / 2)), cc = e / (KC / 2);
        const int64_t row = rb + rr;
        const int col = c0 + cc;
        const double* src = A + (int64_t)col * lda + row;
        const double v0 = (row < r1 && col < n) ? src[0] : 0.0;
        const double v1 = (row + 1 < r1 && col < n) ? src[1] : 0.0;
        E h0, m0, l0, h1, m1, l1;
        LowT<PREC>::split3(v0, h0, m0, l0);
        LowT<PREC>::split3(v1, h1, m1, l1);
        E* dst = lds + cc * LDR + rr;
        *reinterpret_cast<v2bf*>(dst) = v2bf{h0, h1};
        *reinterpret_cast<v2bf*>(dst + PL) = v2bf{m0, m1};
        *reinterpret_cast<v2bf*>(dst + 2 * PL) = v2bf{l0, l1};
      }
    }
    __syncthreads();
    // a wave whose row tiles all lie past the sketch's s rows only helps to stage the chunks
    if (it0 >= it_total) continue;
    if (PREC == TSQR_LOWP_FP32) {
#pragma unroll
      for (int g = 0; g < KC / 16; ++g) {
        const int64_t jbase = rb + 16 * g;
        if (jbase >= r1) break;
        float z[IT][4];
#pragma unroll
        for (int it = 0; it < IT; ++it)
          sketch_normals4((uint64_t)(jbase >> 2) + (uint64_t)q, (uint32_t)((it0 + it) * 16 + c16),
                          k0, k1, z[it]);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          float bop[JT];
#pragma unroll
          for (int jt = 0; jt < JT; ++jt)
            bop[jt] = (float)lds[(16 * jt + c16) * LDR + 16 * g + 4 * q + t];
#pragma unroll
          for (int it = 0; it < IT; ++it)
#pragma unroll
            for (int jt = 0; jt < JT; ++jt) acc[it][jt] = mfma_f32(z[it][t], bop[jt], acc[it][jt]);
        }
      }
    } else {
#pragma unroll
      for (int g = 0; g < KC / 32; ++g) {
        const int64_t jbase = rb + 32 * g;
        if (jbase >= r1) break;
        v8bf a8[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
          float z[8];
          const uint32_t i = (uint32_t)((it0 + it) * 16 + c16);
          const uint64_t p = (uint64_t)(jbase >> 2) + 2 * (uint64_t)q;
          sketch_normals4(p, i, k0, k1, z);
          sketch_normals4(p + 1, i, k0, k1, z + 4);
#pragma unroll
          for (int e = 0; e < 8; ++e) a8[it][e] = (__bf16)z[e];
        }
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) {
          const E* bp = &lds[(16 * jt + c16) * LDR + 32 * g + 8 * q];
          const v8bf bh = *reinterpret_cast<const v8bf*>(bp);
          const v8bf bm = *reinterpret_cast<const v8bf*>(bp + PL);
          const v8bf bl = *reinterpret_cast<const v8bf*>(bp + 2 * PL);
          // smallest terms first
#pragma unroll
          for (int it = 0; it < IT; ++it) {
            acc[it][jt] = mfma_bf16(a8[it], bl, acc[it][jt]);
            acc[it][jt] = mfma_bf16(a8[it], bm, acc[it][jt]);
            acc[it][jt] = mfma_bf16(a8[it], bh, acc[it][jt]);
          }
        }
      }
    }
    // FP32 accumulation over at most 64 rows, then into FP64
#pragma unroll
    for (int it = 0; it < IT; ++it)
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[it][jt][r] += (double)acc[it][jt][r];
        acc[it][jt] = v4f{0.f, 0.f, 0.f, 0.f};
      }
  }

  const size_t Et = (size_t)it_total * jt_total * 256;
  double* dst = part + (size_t)bx * Et;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int itg = it0 + it;
    if (itg >= it_total) continue;
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) {
      const int jtg = bz * JT + jt;
      if (jtg >= jt_total) continue;
      double* tp = dst + ((size_t)itg * jt_total + jtg) * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) tp[lowp_to_f64_tile_index(lane, r)] = acc64[it][jt][r];
    }
  }
}

template <int PREC, int IT, int JT, int NW>
__global__ __launch_bounds__(NW * 64) void k_sketch_lowp(
    int64_t m, int n, const double* __restrict__ A, int64_t lda, uint32_t k0, uint32_t k1,
    int64_t rows_per_block, int it_total, int jt_total, double* __restrict__ part) {
  sketch_lowp_body<PREC, IT, JT, NW>(m, n, A, lda, k0, k1, rows_per_block, it_total, jt_total,
                                     part, (int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z);
}

// Batched form: one work item (problem, row block, i-group, column group) per workgroup;
// the partials have the FP64 sketch's layout, so the batched FP64 reduction sums them.
template <int PREC, int IT, int JT, int NW>
__global__ __launch_bounds__(NW * 64) void k_b_sketch_lowp(const BItem* __restrict__ items,
                                                           const BProb* __restrict__ probs) {
  const BItem it = items[blockIdx.x];
  const BProb& p = probs[it.pid];
  sketch_lowp_body<PREC, IT, JT, NW>(p.m, p.n, p.A, p.lda, p.k0, p.k1, p.sk_rpb, p.sk_it,
                                     p.sk_jt, p.part, it.x, it.y, it.z);
}

// Wide sketch (129..256 columns): every normal is generated once. A workgroup owns NW*IT
// i-tiles (IT per wavefront) and all 16 column tiles of a row block, so the igroups
// workgroups of one row block each read the whole block. They get consecutive slots on
// one XCD (workgroup L runs on XCD L % 8), start together and read the block in the same
// order, so all but one of them find it in that XCD's L2. A is staged through LDS in
// 32-row chunks, the next chunk's loads in flight during the current chunk's products;
// the FP32 accumulators are flushed into FP64 every two chunks (64 rows).
template <int PREC, int NW, int IT>
__global__ __launch_bounds__(NW * 64) void k_sketch_lowp_wide(
    int64_t m, int n, const double* __restrict__ A, int64_t lda, uint32_t k0, uint32_t k1,
    int64_t rows_per_block, int it_total, int jt_total, int igroups, int kblocks,
    double* __restrict__ part) {
  typedef typename LowT<PREC>::E E;
  typedef __attribute__((address_space(1))) const double g_f64;
  constexpr int JT = 16, KC = 32, T = NW * 64;
  constexpr int LDR = KC + (PREC == TSQR_LOWP_FP32 ? 4 : 8);
  constexpr int PF = KC * 16 * JT / T;  // prefetched doubles per thread
  constexpr int PLANES = (PREC == TSQR_LOWP_FP32) ? 1 : 3;  // BF16: hi, mid, lo of A
  constexpr int PL = 16 * JT * LDR;
  __shared__ __attribute__((aligned(16))) E lds[PLANES * PL];

  const int G = kblocks * igroups;
  const int gp8 = (G + 7) / 8;
  const int v = (int)(blockIdx.x % 8) * gp8 + (int)(blockIdx.x / 8);
  if (v >= G) return;  // padding workgroup: exits before any barrier
  const int kb = v / igroups, ig = v % igroups;

  const int lane = lane_id(), wave = wave_id();
  const int q = lane >> 4, c16 = lane & 15;
  const int64_t r0 = (int64_t)kb * rows_per_block;
  const int64_t r1 = min(m, r0 + rows_per_block);
  const int it0 = (ig * NW + wave) * IT;
  // staging: thread t moves rows srow, srow + 1 (srow = 2 (t % 16)) of columns
  // scol + CS k (scol = t / 16, CS = T / 16), k = 0..PF/2-1, and stores each row pair into
  // LDS with one write per plane
  constexpr int CS = T / (KC / 2);
  static_assert(2 * (16 * JT / CS) == PF, "staging map");
  const int srow = 2 * ((int)threadIdx.x % (KC / 2)), scol = (int)threadIdx.x / (KC / 2);

  v4f acc[IT][JT];
  v4d acc64[IT][JT];
#pragma unroll
  for (int ii = 0; ii < IT; ++ii)
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) {
      acc[ii][jt] = v4f{0.f, 0.f, 0.f, 0.f};
      acc64[ii][jt] = v4d{0.0, 0.0, 0.0, 0.0};
    }

  double pf[PF];  // pf[2k], pf[2k+1]: rows srow, srow + 1 of column scol + CS k
  auto fetch = [&](int64_t rb) {
    const int64_t row = rb + srow;
    // a row past the block reads row r0 (the second of a pair whose first row is the
    // block's last reads that row again) and a column past n reads column scol (< n): all
    // valid addresses, zeroed when staged
    g_f64* bp = (g_f64*)(A + (int64_t)scol * lda + (row < r1 ? row : r0));
    g_f64* bp2 = bp + (row + 1 < r1 ? 1 : 0);
    int lim = n - scol;  // column scol + CS k exists iff CS k < lim
    int64_t cstep = (int64_t)CS * lda;  // uniform: the offsets stay scalar per fetch
    asm volatile("" : "+v"(bp), "+v"(bp2), "+v"(lim), "+s"(cstep));
#pragma unroll
    for (int k = 0; k < PF / 2; ++k) {
      const bool ok = CS * k < lim;
      pf[2 * k] = bp[ok ? k * cstep : 0];
      pf[2 * k + 1] = bp2[ok ? k * cstep : 0];
    }
  };
  fetch(r0);
  // 64 rows (two chunks) per iteration, then the flush; a chunk past r1 stages zeros
  for (int64_t rb0 = r0; rb0 < r1; rb0 += 2 * KC) {
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int64_t rb = rb0 + hh * KC;
      __syncthreads();
      {
        const bool rok0 = rb + srow < r1, rok1 = rb + srow + 1 < r1;
#pragma unroll
        for (int k = 0; k < PF / 2; ++k) {
          const int col = scol + CS * k;
          const double v0 = (rok0 && col < n) ? pf[2 * k] : 0.0;
          const double v1 = (rok1 && col < n) ? pf[2 * k + 1] : 0.0;
          E* dst = lds + col * LDR + srow;  // srow and LDR even: a 2-element aligned pair
          if constexpr (PREC == TSQR_LOWP_FP32) {
            *reinterpret_cast<v2f*>(dst) =
                v2f{LowT<PREC>::from_double(v0), LowT<PREC>::from_double(v1)};
          } else {
            E h0, m0, l0, h1, m1, l1;
            LowT<PREC>::split3(v0, h0, m0, l0);
            LowT<PREC>::split3(v1, h1, m1, l1);
            *reinterpret_cast<v2bf*>(dst) = v2bf{h0, h1};
            *reinterpret_cast<v2bf*>(dst + PL) = v2bf{m0, m1};
            *reinterpret_cast<v2bf*>(dst + 2 * PL) = v2bf{l0, l1};
          }
        }
      }
      __syncthreads();
      fetch(rb + KC);  // clamped: always valid addresses
      if constexpr (PREC == TSQR_LOWP_FP32) {
#pragma unroll
        for (int g = 0; g < KC / 16; ++g) {
          float z[IT][4];
#pragma unroll
          for (int ii = 0; ii < IT; ++ii)
            sketch_normals4((uint64_t)((rb + 16 * g) >> 2) + (uint64_t)q,
                            (uint32_t)((it0 + ii) * 16 + c16), k0, k1, z[ii]);
#pragma unroll
          for (int jt = 0; jt < JT; ++jt) {
            typedef __attribute__((address_space(3))) const v4f lds_v4f;
            const v4f b4 = *(lds_v4f*)((__attribute__((address_space(3))) const E*)lds +
                                       (16 * jt + c16) * LDR + 16 * g + 4 * q);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
              for (int ii = 0; ii < IT; ++ii)
                acc[ii][jt] = mfma_f32(z[ii][t], b4[t], acc[ii][jt]);
            // bounded look-ahead of the operand reads (registers)
            if (jt % 4 == 3) __builtin_amdgcn_sched_barrier(0);
          }
        }
      } else {
        v8bf a8[IT];
#pragma unroll
        for (int ii = 0; ii < IT; ++ii) {
          float z[8];
          const uint32_t irow = (uint32_t)((it0 + ii) * 16 + c16);
          const uint64_t p = (uint64_t)(rb >> 2) + 2 * (uint64_t)q;
          sketch_normals4(p, irow, k0, k1, z);
          sketch_normals4(p + 1, irow, k0, k1, z + 4);
#pragma unroll
          for (int e = 0; e < 8; ++e) a8[ii][e] = (__bf16)z[e];
        }
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) {
          typedef __attribute__((address_space(3))) const v8bf lds_v8bf;
          typedef __attribute__((address_space(3))) const E lds_e;
          lds_e* bp = (lds_e*)lds + (16 * jt + c16) * LDR + 8 * q;
          const v8bf bh = *(lds_v8bf*)bp;
          const v8bf bm = *(lds_v8bf*)(bp + PL);
          const v8bf bl = *(lds_v8bf*)(bp + 2 * PL);
          // smallest terms first
#pragma unroll
          for (int ii = 0; ii < IT; ++ii) {
            acc[ii][jt] = mfma_bf16(a8[ii], bl, acc[ii][jt]);
            acc[ii][jt] = mfma_bf16(a8[ii], bm, acc[ii][jt]);
            acc[ii][jt] = mfma_bf16(a8[ii], bh, acc[ii][jt]);
          }
          if (jt % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    // FP32 accumulation over 64 rows, then into FP64
#pragma unroll
    for (int ii = 0; ii < IT; ++ii)
#pragma unroll
      for (int jt = 0; jt < JT; ++jt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[ii][jt][r] += (double)acc[ii][jt][r];
        acc[ii][jt] = v4f{0.f, 0.f, 0.f, 0.f};
      }
  }

#pragma unroll
  for (int ii = 0; ii < IT; ++ii) {
    const int it = it0 + ii;
    double* dst = part + ((size_t)kb * it_total + it) * jt_total * 256;
#pragma unroll
    for (int jt = 0; jt < JT; ++jt)
      if (it < it_total && jt < jt_total)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          dst[(size_t)jt * 256 + lowp_to_f64_tile_index(lane, r)] = acc64[ii][jt][r];
  }
}

// ======================================================== apply A1 = A R0^{-1} ====
// Rinv (n x n upper, FP64) is rounded into the input type and laid out for the A
// operand. FP32: upper 16x16 tiles, tile (a,b) at tri_index(a,b)*256, and inside a tile
// entry (k, c) at c*16 + (k%4)*4 + k/4, so the four K-steps one lane feeds for a tile are
// one 16-byte read. BF16: a padded column-major matrix (ld = rinv_bf16_ld(JT)) so eight
// consecutive k of a column are one 16-byte read.
__host__ __device__ constexpr int lp_tri_index(int a, int b) { return b * (b + 1) / 2 + a; }

// BF16 layout leading dimension: every K-group of 32 rows that a column tile reads must lie
// inside its own column, so ld >= 32 * ceil(jt / 2); the +8 staggers LDS banks.
__host__ __device__ constexpr int rinv_bf16_ld(int jt) { return 32 * ((jt + 1) / 2) + 8; }

template <int PREC>
__host__ __device__ constexpr size_t rinv_elems(int jt) {
  return PREC == TSQR_LOWP_FP32 ? (size_t)jt * (jt + 1) / 2 * 256
                                : (size_t)(16 * jt) * rinv_bf16_ld(jt);
}

template <int PREC>
__global__ void k_rinv_prep(int n, int jt, const double* __restrict__ Rinv, int64_t ldr,
                            typename LowT<PREC>::E* __restrict__ out,
                            const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  const size_t total = rinv_elems<PREC>(jt);
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    int k, c;
    if (PREC == TSQR_LOWP_FP32) {
      const int t = (int)(e / 256), w = (int)(e % 256);
      int b = 0;
      while ((b + 1) * (b + 2) / 2 <= t) ++b;
      const int a = t - b * (b + 1) / 2;
      k = 16 * a + 4 * (w % 4) + (w % 16) / 4;
      c = 16 * b + w / 16;
    } else {
      const int ld = rinv_bf16_ld(jt);
      c = (int)(e / ld);
      k = (int)(e % ld);
    }
    const double v = (k < n && c < n && k <= c) ? Rinv[(int64_t)c * ldr + k] : 0.0;
    out[e] = LowT<PREC>::from_double(v);
  }
}

// One wavefront per 16-row tile; output X = Y Rinv in the input type (column-major).
// Rinv sits once per workgroup in LDS and the workgroup is persistent over the row tiles.
// K-outer order: K-block a of Y (FP32: 16 columns; BF16: a group of 32) adds its products
// to every output block b >= a, after which output block a is final and stored. Only the
// accumulators stay resident; Y streams through a ring of D blocks, each loaded D steps
// ahead (past the tile's last block: the next tile's first blocks), so the loads overlap
// the products of the blocks before them.
// FP32: K-step kk of block a feeds Y(row, 16a + 4kk + q) as the B operand.
// BF16: group g feeds Y(row, 32g + 8q .. 32g + 8q + 7).
// FULL (n == 16 JT, and JT even for BF16): no column bounds. Otherwise a column past n
// loads column 0 of the same row (always a valid address) and is replaced by zero, without
// branches; a row past m loads row 0 and is not stored.
constexpr int kApplyThreads = 1024;

template <int PREC, int JT, bool FULL>
__global__ __launch_bounds__(kApplyThreads) void k_apply_rinv_lowp(
    int64_t m, int n, const double* __restrict__ Y, int64_t ldy,
    const typename LowT<PREC>::E* __restrict__ Ri, typename LowT<PREC>::E* X, int64_t ldx,
    const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  typedef typename LowT<PREC>::E E;
  typedef __attribute__((address_space(1))) const double g_f64;
  typedef __attribute__((address_space(3))) E lds_e;
  constexpr bool F32 = PREC == TSQR_LOWP_FP32;
  constexpr size_t NE = rinv_elems<PREC>(JT);
  constexpr int NK = F32 ? JT : (JT + 1) / 2;  // K-steps: blocks (FP32) or groups (BF16)
  constexpr int CW = F32 ? 16 : 32;            // columns per K-step
  constexpr int PL = F32 ? 4 : 8;              // doubles per lane per K-step
  constexpr int QS = F32 ? 1 : 8;              // lane column stride in q
  constexpr int D = NK < 2 ? NK : 2;           // ring depth (divides NK)
  constexpr int LD = rinv_bf16_ld(JT);
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  E* rl = reinterpret_cast<E*>(smem);
  for (size_t e = threadIdx.x; e < NE; e += blockDim.x) rl[e] = Ri[e];
  __syncthreads();

  const int lane = lane_id();
  const int q = lane >> 4, c16 = lane & 15;
  const int64_t ntiles = (m + 15) / 16;
  const int64_t wstride = (int64_t)gridDim.x * (blockDim.x / kWave);

  // column of element j of K-step k for this lane: CW k + QS q + (F32 ? 4 j : j)
  auto col_of = [&](int k, int j) { return CW * k + QS * q + (F32 ? 4 * j : j); };
  auto load_step = [&](int64_t t, int k, double (&d)[PL]) {
    const int64_t row = t * 16 + c16;
    g_f64* yb = (g_f64*)(Y + (row < m ? row : 0) + (int64_t)(QS * q) * ldy);
    int lim = n - QS * q;  // column c0 + QS q exists iff c0 < lim
    int64_t cstep = ldy;
    asm volatile("" : "+v"(yb), "+v"(lim), "+s"(cstep));
    const int64_t back = -(int64_t)(QS * q) * cstep;  // column 0 of the same row
#pragma unroll
    for (int j = 0; j < PL; ++j) {
      const int c0 = CW * k + (F32 ? 4 * j : j);
      const bool ok = FULL || c0 < lim;
      d[j] = yb[ok ? c0 * cstep : back];
    }
  };

  int64_t tile = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave_id();
  double ring[D][PL];
  if (tile < ntiles) {
#pragma unroll
    for (int k = 0; k < D; ++k) load_step(tile, k, ring[k]);
  }
  for (; tile < ntiles; tile += wstride) {
    const int64_t nxt = tile + wstride < ntiles ? tile + wstride : tile;  // valid address
    const int64_t row = tile * 16 + c16;
    const bool rok = row < m;
    v4f acc[JT];
#pragma unroll
    for (int b = 0; b < JT; ++b) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      // this step's operand in the input type, then its ring slot refilled D steps ahead
      typename std::conditional<F32, v4f, v8bf>::type yv;
#pragma unroll
      for (int j = 0; j < PL; ++j) {
        const bool ok = rok && (FULL || col_of(k, j) < n);
        if constexpr (F32) yv[j] = ok ? (float)ring[k % D][j] : 0.f;
        else yv[j] = LowT<PREC>::from_double(ok ? ring[k % D][j] : 0.0);
      }
      if (k + D < NK) load_step(tile, k + D, ring[k % D]);
      else load_step(nxt, k + D - NK, ring[k % D]);
      if constexpr (F32) {
        lds_e* rp = (lds_e*)rl + c16 * 16 + q * 4;
        asm volatile("" : "+v"(rp));
#pragma unroll
        for (int b = k; b < JT; ++b) {
          typedef __attribute__((address_space(3))) v4f lds_v4f;
          const v4f r4 = *(lds_v4f*)(rp + lp_tri_index(k, b) * 256);
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) acc[b] = mfma_f32(r4[kk], yv[kk], acc[b]);
          if ((b - k) % 4 == 3) __builtin_amdgcn_sched_barrier(0);  // bounded look-ahead
        }
      } else {
        lds_e* rp = (lds_e*)rl + c16 * LD + 8 * q + 32 * k;
        asm volatile("" : "+v"(rp));
#pragma unroll
        for (int b = 2 * k; b < JT; ++b) {
          typedef __attribute__((address_space(3))) v8bf lds_v8bf;
          const v8bf a8 = *(lds_v8bf*)(rp + 16 * b * LD);
          acc[b] = mfma_bf16(a8, yv, acc[b]);
          if ((b - 2 * k) % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
      }
      // output blocks completed by this step: an opaque per-step base and uniform column
      // offsets (the per-lane column products would otherwise be hoisted for all blocks)
      if (rok) {
        E* xb = X + row + (int64_t)(4 * q) * ldx;
        int64_t xs = ldx;
        asm volatile("" : "+v"(xb), "+s"(xs));
#pragma unroll
        for (int b = F32 ? k : 2 * k; b < (F32 ? k + 1 : 2 * k + 2) && b < JT; ++b)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (FULL || 16 * b + 4 * q + r < n)
              xb[(16 * b + r) * xs] = LowT<PREC>::from_float(acc[b][r]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

// ================================================================= Gram (low) ====
// W partials (FP64, tile-native) of X^T X for X in the input type.  A workgroup streams
// its row block in 64-row chunks, the next chunk loaded into registers (16-byte loads)
// while the current one, staged in LDS, feeds the matrix cores (FP32: row-major LDS, one
// K-step per 4 rows; BF16: column-major LDS so that eight consecutive rows are one
// 16-byte read, one K-step per 32 rows).  FP32 accumulation over each 64-row chunk, then
// into FP64 registers.  The upper tiles are shared out over NS workgroups per row block
// (blockIdx.y) and NW waves each: slot y NW + w owns tiles t = slot, slot + NS NW, ...;
// the tile set is a compile-time property of the slot.
template <int PREC>
struct LowOp;
template <>
struct LowOp<TSQR_LOWP_FP32> {
  typedef float T;
  static __device__ __forceinline__ v4f mma(T a, T b, v4f c) { return mfma_f32(a, b, c); }
};
template <>
struct LowOp<TSQR_LOWP_BF16> {
  typedef v8bf T;
  static __device__ __forceinline__ v4f mma(T a, T b, v4f c) { return mfma_bf16(a, b, c); }
};

template <int PREC, int STRIDE, int SLOT, int TPW, int... U>
__device__ __forceinline__ void gram_lowp_step(const typename LowOp<PREC>::T* op, v4f (&acc)[TPW],
                                               std::integer_sequence<int, U...>) {
  ((acc[U] = LowOp<PREC>::mma(op[UpperTile<SLOT + U * STRIDE>::a],
                              op[UpperTile<SLOT + U * STRIDE>::b], acc[U])),
   ...);
}

template <int PREC, int JT, int STRIDE, int SLOT, int KC, int LDA, int TPW>
__device__ __forceinline__ void gram_lowp_chunk(const typename LowT<PREC>::E* lds, int q,
                                                int c16, v4f (&acc)[TPW]) {
  constexpr int NT = JT * (JT + 1) / 2;
  constexpr int CNT = NT > SLOT ? (NT - SLOT + STRIDE - 1) / STRIDE : 0;
  typedef typename LowT<PREC>::E E;
  typedef __attribute__((address_space(3))) const E lds_e;
  if constexpr (PREC == TSQR_LOWP_FP32) {
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      // opaque per-step row pointer: keeps each step's operand reads next to its MFMAs
      lds_e* rowp = (lds_e*)(lds + (4 * kk + q) * LDA + c16);
      asm volatile("" : "+v"(rowp));
      float op[JT];
#pragma unroll
      for (int c = 0; c < JT; ++c) op[c] = rowp[16 * c];
      gram_lowp_step<PREC, STRIDE, SLOT, TPW>(op, acc, std::make_integer_sequence<int, CNT>{});
    }
  } else {
#pragma unroll
    for (int g = 0; g < KC / 32; ++g) {
      v8bf op[JT];
#pragma unroll
      for (int c = 0; c < JT; ++c)
        op[c] = *reinterpret_cast<const v8bf*>(&lds[(16 * c + c16) * LDA + 32 * g + 8 * q]);
      gram_lowp_step<PREC, STRIDE, SLOT, TPW>(op, acc, std::make_integer_sequence<int, CNT>{});
    }
  }
}

// VEC: X is 16-byte aligned and ldx, m are multiples of the elements per 16-byte word
// (chosen on the host), so every in-range row group is one aligned load; the loads are
// branch-free either way.
template <int PREC, int JT, int NW, int NS, bool VEC>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(2))) void k_gram_lowp(int64_t m, int n,
                                                       const typename LowT<PREC>::E* __restrict__ X,
                                                       int64_t ldx, int64_t rows_per_block,
                                                       int ntiles, double* __restrict__ part,
                                                       const int* __restrict__ gate) {
  if (gate && *gate == 0) return;  // gated off on the device
  typedef typename LowT<PREC>::E E;
  constexpr bool F32 = PREC == TSQR_LOWP_FP32;
  constexpr int KC = 64;
  constexpr int NC = JT * 16;
  constexpr int NT = JT * (JT + 1) / 2;
  constexpr int STRIDE = NW * NS;
  constexpr int TPW = (NT + STRIDE - 1) / STRIDE;
  constexpr int THREADS = NW * 64;
  constexpr int EPL = 16 / sizeof(E);        // elements per 16-byte load (rows of a column)
  constexpr int RPC = KC / EPL;              // loads per column per chunk
  constexpr int CPP = THREADS / RPC;         // columns per pass
  constexpr int PASSES = (NC + CPP - 1) / CPP;
  constexpr int LDA = F32 ? NC + 1 : KC + 8;  // row-major / column-major
  static_assert(STRIDE <= 16, "slot dispatch covers at most 16 slots");
  __shared__ __attribute__((aligned(16))) E lds[F32 ? KC * LDA : NC * LDA];

  const int lane = lane_id(), wave = wave_id();
  const int q = lane >> 4, c16 = lane & 15;
  const int slot = (int)blockIdx.y * NW + wave;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(m, r0 + rows_per_block);
  v4f acc[TPW];
  v4d acc64[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
    acc64[u] = v4d{0.0, 0.0, 0.0, 0.0};
  }

  // rows start at multiples of 64; with m a multiple of EPL, row < r1 implies that the
  // whole group row .. row + EPL - 1 is in range
  const int rp = (int)threadIdx.x % RPC, cb = (int)threadIdx.x / RPC;
  E pre[PASSES][EPL];
  auto load_chunk = [&](int64_t rb) {
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
      const int cc = cb + ps * CPP;
      const int64_t row = rb + EPL * rp;
      const bool okc = (cc < NC) && (cc < n);
      if constexpr (VEC) {
        const bool ok = okc && row < r1;
        const E* src = ok ? X + (int64_t)cc * ldx + row : X;  // clamped, always valid
        uint4 v = *reinterpret_cast<const uint4*>(src);
        if (!ok) v = uint4{0u, 0u, 0u, 0u};
        __builtin_memcpy(pre[ps], &v, 16);
      } else {
        const E* src = X + (int64_t)cc * ldx + row;
#pragma unroll
        for (int e = 0; e < EPL; ++e)
          pre[ps][e] = (okc && row + e < r1) ? src[e] : LowT<PREC>::from_float(0.f);
      }
    }
  };

  if (r0 < r1) load_chunk(r0);
  for (int64_t rb = r0; rb < r1; rb += KC) {
    __syncthreads();
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
      const int cc = cb + ps * CPP;
      if (cc < NC) {
        if constexpr (F32) {
#pragma unroll
          for (int e = 0; e < EPL; ++e) lds[(EPL * rp + e) * LDA + cc] = pre[ps][e];
        } else {
          *reinterpret_cast<uint4*>(&lds[cc * LDA + EPL * rp]) =
              *reinterpret_cast<const uint4*>(pre[ps]);
        }
      }
    }
    __syncthreads();
    if (rb + KC < r1) load_chunk(rb + KC);
    switch (slot) {
#define TSQR_GRL_SLOT(S_)                                                                   \
  case S_:                                                                                  \
    if constexpr (S_ < STRIDE)                                                              \
      gram_lowp_chunk<PREC, JT, STRIDE, S_, KC, LDA, TPW>(lds, q, c16, acc);                \
    break;
      TSQR_GRL_SLOT(0) TSQR_GRL_SLOT(1) TSQR_GRL_SLOT(2) TSQR_GRL_SLOT(3)
      TSQR_GRL_SLOT(4) TSQR_GRL_SLOT(5) TSQR_GRL_SLOT(6) TSQR_GRL_SLOT(7)
      TSQR_GRL_SLOT(8) TSQR_GRL_SLOT(9) TSQR_GRL_SLOT(10) TSQR_GRL_SLOT(11)
      TSQR_GRL_SLOT(12) TSQR_GRL_SLOT(13) TSQR_GRL_SLOT(14) TSQR_GRL_SLOT(15)
#undef TSQR_GRL_SLOT
      default: break;
    }
#pragma unroll
    for (int u = 0; u < TPW; ++u) {
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[u][r] += (double)acc[u][r];
      acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  }
  double* dst = part + (size_t)blockIdx.x * ntiles * 256;
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int t = slot + u * STRIDE;
    if (t < NT && t < ntiles)
#pragma unroll
      for (int r = 0; r < 4; ++r) dst[(size_t)t * 256 + lowp_to_f64_tile_index(lane, r)] = acc64[u][r];
  }
}

// ================================================================== launchers ====
static int jt_pow2(int n) {
  int jt = 1;
  while (jt < (n + 15) / 16) jt <<= 1;
  return jt;
}

size_t lowp_elem_bytes(int prec) { return prec == TSQR_LOWP_FP32 ? 4 : 2; }

size_t rinv_lowp_bytes(int prec, int n) {
  const int jt = jt_pow2(n);
  return (prec == TSQR_LOWP_FP32 ? rinv_elems<TSQR_LOWP_FP32>(jt) * 4
                                 : rinv_elems<TSQR_LOWP_BF16>(jt) * 2);
}

template <int PREC, int IT, int JT, int NW>
static hipError_t sketch_lowp_t(const SketchPlan& p, int64_t m, int n, const double* A,
                                int64_t lda, uint64_t seed, double* part, hipStream_t st) {
  dim3 grid(p.kblocks, p.igroups, p.jgroups);
  hipLaunchKernelGGL((k_sketch_lowp<PREC, IT, JT, NW>), grid, dim3(NW * 64), 0, st, m, n, A, lda,
                     (uint32_t)seed, (uint32_t)(seed >> 32), p.rows_per_block, p.it_total,
                     p.jt_total, part);
  return hipGetLastError();
}

#ifndef TSQR_SKW_NW
#define TSQR_SKW_NW 8
#define TSQR_SKW_IT 1
#endif
constexpr int kSkwNW = TSQR_SKW_NW, kSkwIT = TSQR_SKW_IT;

hipError_t launch_sketch_lowp(int prec, const SketchPlan& p, int64_t m, int n, const double* A,
                              int64_t lda, uint64_t seed, double* part, hipStream_t st) {
  if (p.jt_total > 8) {
    // all columns per workgroup; same row blocks (and partial layout) as the plan
    constexpr int NW = kSkwNW, IT = kSkwIT;
    const int igroups = (p.it_total + NW * IT - 1) / (NW * IT);
    const int G = p.kblocks * igroups;
    const dim3 grid((unsigned)((G + 7) / 8 * 8)), block(NW * 64);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    if (prec == TSQR_LOWP_FP32)
      hipLaunchKernelGGL((k_sketch_lowp_wide<TSQR_LOWP_FP32, NW, IT>), grid, block, 0, st, m, n,
                         A, lda, k0, k1, p.rows_per_block, p.it_total, p.jt_total, igroups,
                         p.kblocks, part);
    else
      hipLaunchKernelGGL((k_sketch_lowp_wide<TSQR_LOWP_BF16, NW, IT>), grid, block, 0, st, m, n,
                         A, lda, k0, k1, p.rows_per_block, p.it_total, p.jt_total, igroups,
                         p.kblocks, part);
    return hipGetLastError();
  }
  // the FP64 sketch's 16-wavefront shape (one row tile each) runs here as 8 wavefronts of
  // two row tiles: the same 16 row tiles per workgroup, row blocks and partial layout
  SketchPlan q = p;
  if (q.NW == 16 && q.IT == 1) {
    q.NW = 8;
    q.IT = 2;
  }
#define TSQR_SKL(PR, IT_, JT_, NW_)                                                           \
  if (prec == PR && q.IT == IT_ && q.JT == JT_ && q.NW == NW_)                                \
    return sketch_lowp_t<PR, IT_, JT_, NW_>(q, m, n, A, lda, seed, part, st);
#define TSQR_SKL_ALL(PR)                                                                      \
  TSQR_SKL(PR, 1, 1, 4) TSQR_SKL(PR, 1, 2, 4) TSQR_SKL(PR, 1, 4, 4) TSQR_SKL(PR, 1, 8, 4)     \
  TSQR_SKL(PR, 1, 1, 8) TSQR_SKL(PR, 1, 2, 8) TSQR_SKL(PR, 1, 4, 8) TSQR_SKL(PR, 1, 8, 8)     \
  TSQR_SKL(PR, 2, 8, 4) TSQR_SKL(PR, 2, 8, 8) TSQR_SKL(PR, 2, 4, 8) TSQR_SKL(PR, 2, 4, 4)     \
  TSQR_SKL(PR, 2, 2, 8) TSQR_SKL(PR, 2, 1, 8) TSQR_SKL(PR, 2, 2, 4) TSQR_SKL(PR, 2, 1, 4)
  TSQR_SKL_ALL(TSQR_LOWP_FP32)
  TSQR_SKL_ALL(TSQR_LOWP_BF16)
#undef TSQR_SKL_ALL
#undef TSQR_SKL
  return hipErrorInvalidValue;
}

hipError_t launch_rinv_prep(int prec, int n, const double* Rinv, int64_t ldr, void* out,
                            hipStream_t st, const int* gate) {
  const int jt = jt_pow2(n);
  if (jt > 16) return hipErrorInvalidValue;
  const size_t total = prec == TSQR_LOWP_FP32 ? rinv_elems<TSQR_LOWP_FP32>(jt)
                                              : rinv_elems<TSQR_LOWP_BF16>(jt);
  int blocks = (int)((total + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  if (prec == TSQR_LOWP_FP32)
    hipLaunchKernelGGL(k_rinv_prep<TSQR_LOWP_FP32>, dim3(blocks), dim3(256), 0, st, n, jt, Rinv,
                       ldr, (float*)out, gate);
  else
    hipLaunchKernelGGL(k_rinv_prep<TSQR_LOWP_BF16>, dim3(blocks), dim3(256), 0, st, n, jt, Rinv,
                       ldr, (__bf16*)out, gate);
  return hipGetLastError();
}

hipError_t launch_apply_rinv_lowp(int prec, int64_t m, int n, const double* Y, int64_t ldy,
                                  const void* Ri, void* X, int64_t ldx, hipStream_t st,
                                  const int* gate) {
  const int jt = jt_pow2(n);
  const int64_t ntiles = (m + 15) / 16;
  const int nt = kApplyThreads;
  int64_t blocks = (ntiles + nt / kWave - 1) / (nt / kWave);
  const int64_t cap = (int64_t)device_cu_count();  // one workgroup (and one Rinv copy) per CU
  if (blocks > cap) blocks = cap;
  dim3 grid((unsigned)blocks), block(nt);
  // FULL drops the column bounds: every column a K-step reads must exist (BF16 reads whole
  // 32-column groups, so a single 16-column tile never qualifies)
  const bool full = n == 16 * jt && (prec == TSQR_LOWP_FP32 || jt % 2 == 0);
#define TSQR_APL(PR, J)                                                                        \
  if (prec == PR && jt == J) {                                                                 \
    typedef typename LowT<PR>::E E;                                                            \
    const size_t sh = rinv_elems<PR>(J) * sizeof(E);                                           \
    if (full)                                                                                  \
      hipLaunchKernelGGL((k_apply_rinv_lowp<PR, J, true>), grid, block, sh, st, m, n, Y, ldy,   \
                         (const E*)Ri, (E*)X, ldx, gate);                                      \
    else                                                                                       \
      hipLaunchKernelGGL((k_apply_rinv_lowp<PR, J, false>), grid, block, sh, st, m, n, Y, ldy,  \
                         (const E*)Ri, (E*)X, ldx, gate);                                      \
    return hipGetLastError();                                                                  \
  }
  TSQR_APL(TSQR_LOWP_FP32, 1) TSQR_APL(TSQR_LOWP_FP32, 2) TSQR_APL(TSQR_LOWP_FP32, 4)
  TSQR_APL(TSQR_LOWP_FP32, 8) TSQR_APL(TSQR_LOWP_FP32, 16)
  TSQR_APL(TSQR_LOWP_BF16, 1) TSQR_APL(TSQR_LOWP_BF16, 2) TSQR_APL(TSQR_LOWP_BF16, 4)
  TSQR_APL(TSQR_LOWP_BF16, 8) TSQR_APL(TSQR_LOWP_BF16, 16)
#undef TSQR_APL
  return hipErrorInvalidValue;
}

hipError_t launch_b_sketch_lowp(int prec, int IT, int JT, int NW, const BItem* items, int nitems,
                                const BProb* probs, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
#define TSQR_BSKL(PR, IT_, JT_, NW_)                                                            \
  if (prec == PR && IT == IT_ && JT == JT_ && NW == NW_) {                                     \
    hipLaunchKernelGGL((k_b_sketch_lowp<PR, IT_, JT_, NW_>), dim3(nitems), dim3(NW_ * 64), 0,   \
                       st, items, probs);                                                      \
    return hipGetLastError();                                                                  \
  }
#define TSQR_BSKL_ALL(PR)                                                                      \
  TSQR_BSKL(PR, 1, 1, 4) TSQR_BSKL(PR, 1, 2, 4) TSQR_BSKL(PR, 1, 4, 4) TSQR_BSKL(PR, 1, 8, 4) \
  TSQR_BSKL(PR, 1, 1, 8) TSQR_BSKL(PR, 1, 2, 8) TSQR_BSKL(PR, 1, 4, 8) TSQR_BSKL(PR, 1, 8, 8) \
  TSQR_BSKL(PR, 2, 8, 4) TSQR_BSKL(PR, 2, 8, 8) TSQR_BSKL(PR, 2, 4, 8) TSQR_BSKL(PR, 2, 4, 4) \
  TSQR_BSKL(PR, 2, 2, 8) TSQR_BSKL(PR, 2, 1, 8) TSQR_BSKL(PR, 2, 2, 4) TSQR_BSKL(PR, 2, 1, 4)
  TSQR_BSKL_ALL(TSQR_LOWP_FP32)
  TSQR_BSKL_ALL(TSQR_LOWP_BF16)
#undef TSQR_BSKL_ALL
#undef TSQR_BSKL
  return hipErrorInvalidValue;
}

hipError_t launch_gram_lowp(int prec, const GramPlan& p, int64_t m, int n, const void* X,
                            int64_t ldx, double* part, hipStream_t st, const int* gate) {
  const int64_t epl = prec == TSQR_LOWP_FP32 ? 4 : 8;
  const bool vec = ((reinterpret_cast<uintptr_t>(X) & 15) == 0) && (ldx % epl == 0) &&
                   (m % epl == 0);
#define TSQR_GRL(PR, J, NW_, NS_)                                                             \
  if (prec == PR && p.jt_total <= J) {                                                        \
    typedef typename LowT<PR>::E E;                                                           \
    if (vec)                                                                                  \
      hipLaunchKernelGGL((k_gram_lowp<PR, J, NW_, NS_, true>), dim3(p.kblocks, NS_),           \
                         dim3(NW_ * 64), 0, st, m, n, (const E*)X, ldx, p.rows_per_block,      \
                         p.ntiles, part, gate);                                               \
    else                                                                                      \
      hipLaunchKernelGGL((k_gram_lowp<PR, J, NW_, NS_, false>), dim3(p.kblocks, NS_),          \
                         dim3(NW_ * 64), 0, st, m, n, (const E*)X, ldx, p.rows_per_block,      \
                         p.ntiles, part, gate);                                               \
    return hipGetLastError();                                                                 \
  }
  TSQR_GRL(TSQR_LOWP_FP32, 1, 4, 1) TSQR_GRL(TSQR_LOWP_FP32, 2, 4, 1)
  TSQR_GRL(TSQR_LOWP_FP32, 4, 4, 1) TSQR_GRL(TSQR_LOWP_FP32, 8, 4, 1)
  TSQR_GRL(TSQR_LOWP_FP32, 16, 8, 2)
  TSQR_GRL(TSQR_LOWP_BF16, 1, 4, 1) TSQR_GRL(TSQR_LOWP_BF16, 2, 4, 1)
  TSQR_GRL(TSQR_LOWP_BF16, 4, 4, 1) TSQR_GRL(TSQR_LOWP_BF16, 8, 4, 1)
  TSQR_GRL(TSQR_LOWP_BF16, 16, 8, 2)
#undef TSQR_GRL
  return hipErrorInvalidValue;
}

}  // namespace tsqr
