// Gaussian sketch B = S A (paper Section 2.3, Gaussian ensemble) on FP64 MFMA.
//
// S = Z / sqrt(s) is never stored: every lane regenerates the entries of Z it feeds to
// the matrix cores from the Philox4x32-10 stream.  The GEMM is split over row blocks of A
// (split-K); each workgroup writes one partial s x n sum, and a second kernel adds the
// partials in a fixed order, so the result is bitwise reproducible run to run.
//
// MFMA mapping (16x16x4 FP64, see tsqr_device.hpp): for a 16-row group of A starting at
// row j0, K-step t uses MFMA k-index q = lane/16 for row j0 + 4q + t.  Lane l therefore
// needs Z(i, j0+4q .. j0+4q+3) for one i = i-tile base + l%16: exactly the four normals
// of one Philox call (counter p = j0/4 + q), so no normal is generated twice.
#include "tsqr_device.hpp"
#include "tsqr_launch.hpp"

namespace tsqr {

// Body of one workgroup: row block bx, i-tile group by, column group bz (the kernel's
// blockIdx; the batched kernels supply them from their work lists).  EXTL: the LDS chunk
// buffers live at ext_lds (sketch_f64_lds_doubles<JT>() doubles, provided by a kernel that
// hosts several bodies) instead of in the body's own LDS.
template <int JT>
__host__ __device__ constexpr int sketch_f64_lds_doubles() {
  return 2 * 32 * (JT * 16 + 1);
}

template <int IT, int JT, int NW, bool EXTL = false>
__device__ __forceinline__ void sketch_f64_body(int64_t m, int n, const double* __restrict__ A,
                                                int64_t lda, uint32_t k0, uint32_t k1,
                                                int64_t rows_per_block, int it_total,
                                                int jt_total, double* __restrict__ part, int bx,
                                                int by, int bz, double* ext_lds = nullptr) {
  constexpr int KC = 32;          // rows of A per LDS chunk
  constexpr int NC = JT * 16;     // columns of A per workgroup
  constexpr int LDN = NC + 1;     // padded row length of the LDS chunk (doubles)
  constexpr int T = NW * 64;      // threads
  constexpr int CPP = T / (KC / 2);                 // columns loaded per pass
  constexpr int PASSES = (NC + CPP - 1) / CPP;
  // double buffer: one barrier per chunk
  double* lbase;
  if constexpr (EXTL) {
    lbase = ext_lds;
  } else {
    __shared__ double own[2 * KC * LDN];
    lbase = own;
  }
  double(*ldsb)[KC * LDN] = reinterpret_cast<double(*)[KC * LDN]>(lbase);

  const int lane = lane_id(), wave = wave_id();
  const int q = lane >> 4, c16 = lane & 15;
  const int64_t r0 = (int64_t)bx * rows_per_block;
  const int64_t r1 = min(m, r0 + rows_per_block);
  const int it0 = by * (NW * IT) + wave * IT;
  const int c0 = bz * NC;

  v4d acc[IT][JT];
#pragma unroll
  for (int it = 0; it < IT; ++it)
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) acc[it][jt] = v4d{0.0, 0.0, 0.0, 0.0};

  // cooperative loader: thread handles rows (2rp, 2rp+1) of columns cb + pass*CPP
  const int rp = (int)threadIdx.x % (KC / 2), cb = (int)threadIdx.x / (KC / 2);
  double pre[PASSES][2];
  auto load_chunk = [&](int64_t rb) {
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
      const int cc = cb + ps * CPP;
      const int col = c0 + cc;
      const int64_t row = rb + 2 * rp;
      const bool okc = (cc < NC) && (col < n);
      const double* src = A + (int64_t)col * lda + row;
      pre[ps][0] = (okc && row < r1) ? src[0] : 0.0;
      pre[ps][1] = (okc && row + 1 < r1) ? src[1] : 0.0;
    }
  };
  auto store_chunk = [&](double* lds) {
#pragma unroll
    for (int ps = 0; ps < PASSES; ++ps) {
      const int cc = cb + ps * CPP;
      if (cc < NC) {
        lds[(2 * rp) * LDN + cc] = pre[ps][0];
        lds[(2 * rp + 1) * LDN + cc] = pre[ps][1];
      }
    }
  };

  if (r0 < r1) {
    load_chunk(r0);
    store_chunk(ldsb[0]);
    if (r0 + KC < r1) load_chunk(r0 + KC);
  }
  __syncthreads();
  int cur = 0;
  // a wave whose row tiles all lie past the sketch's s rows (a workgroup wider than B)
  // only helps to stage the chunks
  const bool active = it0 < it_total;
  for (int64_t rb = r0; rb < r1; rb += KC, cur ^= 1) {
    const double* lds = ldsb[cur];
#pragma unroll
    for (int g = 0; g < KC / 16; ++g) {
      const int64_t jbase = rb + 16 * g;
      if (jbase >= r1 || !active) break;
      float z[IT][4];
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const uint32_t i = (uint32_t)((it0 + it) * 16 + c16);
        const uint64_t p = (uint64_t)(jbase >> 2) + (uint64_t)q;
        sketch_normals4(p, i, k0, k1, z[it]);
      }
      // raised issue priority while this wave feeds the matrix core, so that the arbiter
      // prefers MFMA issue over other waves' normal generation (measured: 2^20 x 128,
      // 1.173 -> 1.162 ms; 2^20 x 64, 0.389 -> 0.374 ms)
      __builtin_amdgcn_s_setprio(1);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double bop[JT];
#pragma unroll
        for (int jt = 0; jt < JT; ++jt) bop[jt] = lds[(16 * g + 4 * q + t) * LDN + 16 * jt + c16];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
          const double a = (double)z[it][t];
#pragma unroll
          for (int jt = 0; jt < JT; ++jt) acc[it][jt] = mfma_f64(a, bop[jt], acc[it][jt]);
        }
      }
      __builtin_amdgcn_s_setprio(0);
    }
    if (rb + KC < r1) store_chunk(ldsb[cur ^ 1]);
    __syncthreads();
    if (rb + 2 * KC < r1) load_chunk(rb + 2 * KC);
  }

  const size_t E = (size_t)it_total * (size_t)jt_total * 256;
  double* dst = part + (size_t)bx * E;
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int itg = it0 + it;
    if (itg >= it_total) continue;
#pragma unroll
    for (int jt = 0; jt < JT; ++jt) {
      const int jtg = bz * JT + jt;
      if (jtg >= jt_total) continue;
      double* tp = dst + ((size_t)itg * jt_total + jtg) * 256 + lane * 4;
      *reinterpret_cast<v4d*>(tp) = acc[it][jt];
    }
  }
}

template <int IT, int JT, int NW>
__global__ __launch_bounds__(NW * 64) void k_sketch_f64(
    int64_t m, int n, const double* __restrict__ A, int64_t lda, uint32_t k0, uint32_t k1,
    int64_t rows_per_block, int it_total, int jt_total, double* __restrict__ part) {
  sketch_f64_body<IT, JT, NW>(m, n, A, lda, k0, k1, rows_per_block, it_total, jt_total, part,
                              (int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z);
}

// B(i, c) = scale * sum_kb part[kb][tile(i,c)][lane][reg].  A 256-thread block handles 16
// consecutive partial entries; thread group g (16 of them) sums the row blocks kb = g,
// g+16, ... in increasing order and the 16 group sums are added in group order, so the
// result does not depend on timing (deterministic).
__device__ __forceinline__ void sketch_reduce_body(int kblocks, int it_total, int jt_total, int s,
                                                   int n, const double* __restrict__ part,
                                                   double scale, double* __restrict__ B,
                                                   int64_t ldb, int bx) {
  __shared__ double red[16][17];
  const size_t E = (size_t)it_total * jt_total * 256;
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
    const int itg = tile / jt_total, jtg = tile % jt_total;
    const int i = 16 * itg + 4 * r + (lane >> 4), c = 16 * jtg + (lane & 15);
    if (i < s && c < n) B[(int64_t)c * ldb + i] = scale * t;
  }
}

__global__ __launch_bounds__(256) void k_sketch_reduce(int kblocks, int it_total, int jt_total,
                                                       int s, int n,
                                                       const double* __restrict__ part,
                                                       double scale, double* __restrict__ B,
                                                       int64_t ldb) {
  sketch_reduce_body(kblocks, it_total, jt_total, s, n, part, scale, B, ldb, (int)blockIdx.x);
}

// --- batched forms ------------------------------------------------------------------------
template <int IT, int JT, int NW>
__global__ __launch_bounds__(NW * 64) void k_b_sketch(const BItem* __restrict__ items,
                                                      const BProb* __restrict__ probs) {
  const BItem it = items[blockIdx.x];
  const BProb& p = probs[it.pid];
  sketch_f64_body<IT, JT, NW>(p.m, p.n, p.A, p.lda, p.k0, p.k1, p.sk_rpb, p.sk_it, p.sk_jt, p.part,
                              it.x, it.y, it.z);
}

__global__ __launch_bounds__(256) void k_b_sketch_reduce(const BItem* __restrict__ items,
                                                         const BProb* __restrict__ probs) {
  const BItem it = items[blockIdx.x];
  const BProb& p = probs[it.pid];
  sketch_reduce_body(p.sk_kblocks, p.sk_it, p.sk_jt, p.s, p.n, p.part, p.scale, p.B, p.s, it.x);
}

// --- debug / test kernels --------------------------------------------------------------
__global__ void k_philox_words(int64_t count, const uint32_t* __restrict__ ctr, uint32_t k0,
                               uint32_t k1, uint32_t* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const U32x4 w = philox4x32_10(U32x4{ctr[4 * e], ctr[4 * e + 1], ctr[4 * e + 2], ctr[4 * e + 3]},
                                  k0, k1);
    out[4 * e] = w.x;
    out[4 * e + 1] = w.y;
    out[4 * e + 2] = w.z;
    out[4 * e + 3] = w.w;
  }
}

__global__ void k_sketch_normals(uint32_t k0, uint32_t k1, int64_t i0, int64_t ni, int64_t j0,
                                 int64_t nj, double* __restrict__ Z, int64_t ldz) {
  const int64_t total = ni * nj;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = e % ni, b = e / ni;
    const int64_t j = j0 + b;
    float z[4];
    sketch_normals4((uint64_t)j >> 2, (uint32_t)(i0 + a), k0, k1, z);
    Z[b * ldz + a] = (double)z[j & 3];
  }
}

// --- planning and launch -------------------------------------------------------------
SketchPlan plan_sketch(int64_t m, int n, int s) {
  SketchPlan p{};
  p.it_total = (s + 15) / 16;
  p.jt_total = (n + 15) / 16;
  p.JT = p.jt_total >= 8 ? 8 : (p.jt_total >= 4 ? 4 : (p.jt_total >= 2 ? 2 : 1));
  p.jgroups = (p.jt_total + p.JT - 1) / p.JT;
  p.IT = p.it_total >= 16 ? 2 : 1;
  const int waves_needed = (p.it_total + p.IT - 1) / p.IT;
  p.NW = waves_needed >= 8 ? 8 : 4;
  // at least 16 row tiles and 8 column tiles: sixteen wavefronts of one row tile each (four
  // per SIMD, within 128 registers) hide latency better than eight with two (measured:
  // 2^20 x 128, s = 256: 1.268 -> 1.259 ms; 2^20 x 256, s = 512: 4.74 -> 4.61 ms); every
  // tile is still summed by one wavefront over the same rows, so B does not change
  if (p.it_total >= 16 && p.JT == 8) {
    p.IT = 1;
    p.NW = 16;
  }
  p.igroups = (p.it_total + p.NW * p.IT - 1) / (p.NW * p.IT);
  const int cus = device_cu_count();
  // one workgroup of 8 or 16 wavefronts (or two 4-wave ones) per compute unit
  int64_t target = (int64_t)cus * (p.NW >= 8 ? 1 : 2) / (p.igroups * p.jgroups);
  if (target < 1) target = 1;
  int64_t rpb = (m + target - 1) / target;
  rpb = ((rpb + 31) / 32) * 32;
  if (rpb < 32) rpb = 32;
  p.rows_per_block = rpb;
  p.kblocks = (int)((m + rpb - 1) / rpb);
  if (p.kblocks < 1) p.kblocks = 1;
  p.part_doubles = (size_t)p.kblocks * p.it_total * p.jt_total * 256;
  return p;
}

template <int IT, int JT, int NW>
static hipError_t launch_sketch_t(const SketchPlan& p, int64_t m, int n, const double* A,
                                  int64_t lda, uint32_t k0, uint32_t k1, double* part,
                                  hipStream_t st) {
  dim3 grid(p.kblocks, p.igroups, p.jgroups);
  hipLaunchKernelGGL((k_sketch_f64<IT, JT, NW>), grid, dim3(NW * 64), 0, st, m, n, A, lda, k0,
                     k1, p.rows_per_block, p.it_total, p.jt_total, part);
  return hipGetLastError();
}

hipError_t launch_sketch(const SketchPlan& p, int64_t m, int n, const double* A, int64_t lda,
                         int s, uint64_t seed, double* part, hipStream_t st) {
  (void)s;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#define TSQR_SK(IT_, JT_, NW_)                                                         \
  if (p.IT == IT_ && p.JT == JT_ && p.NW == NW_)                                       \
    return launch_sketch_t<IT_, JT_, NW_>(p, m, n, A, lda, k0, k1, part, st);
  TSQR_SK(1, 1, 4) TSQR_SK(1, 2, 4) TSQR_SK(1, 4, 4) TSQR_SK(1, 8, 4)
  TSQR_SK(1, 1, 8) TSQR_SK(1, 2, 8) TSQR_SK(1, 4, 8) TSQR_SK(1, 8, 8)
  TSQR_SK(2, 8, 4) TSQR_SK(2, 8, 8) TSQR_SK(2, 4, 8) TSQR_SK(2, 4, 4)
  TSQR_SK(2, 2, 8) TSQR_SK(2, 1, 8) TSQR_SK(2, 2, 4) TSQR_SK(2, 1, 4) TSQR_SK(1, 8, 16)
#undef TSQR_SK
  return hipErrorInvalidValue;
}

// Row-extraction sketch (the sketch of the paper's experiments, Section 2.3), sampled as in
// Theorem "Equal Probability Case": draw i picks row r_i = floor(w m / 2^64) for the 64-bit
// word w = x + 2^32 y of Philox4x32-10 with counter (i lo, i hi, 0, 1) (the last counter
// word is 0 in every Gaussian-sketch call, so the two streams never meet), independently
// of the other draws; B(i, :) = A(r_i, :).  One workgroup per draw, columns over threads.
__global__ __launch_bounds__(256) void k_sketch_rows(int64_t m, int n,
                                                     const double* __restrict__ A, int64_t lda,
                                                     uint32_t k0, uint32_t k1,
                                                     double* __restrict__ B, int64_t ldb) {
  const uint64_t i = blockIdx.x;
  const U32x4 w = philox4x32_10(U32x4{(uint32_t)i, (uint32_t)(i >> 32), 0u, 1u}, k0, k1);
  const uint64_t w64 = (uint64_t)w.x | ((uint64_t)w.y << 32);
  const int64_t r = (int64_t)__umul64hi(w64, (uint64_t)m);  // in [0, m)
  for (int j = threadIdx.x; j < n; j += blockDim.x)
    B[(int64_t)j * ldb + (int64_t)i] = A[(int64_t)j * lda + r];
}

hipError_t launch_sketch_rows(int64_t m, int n, const double* A, int64_t lda, int s,
                              uint64_t seed, double* B, int64_t ldb, hipStream_t st) {
  hipLaunchKernelGGL(k_sketch_rows, dim3(s), dim3(256), 0, st, m, n, A, lda, (uint32_t)seed,
                     (uint32_t)(seed >> 32), B, ldb);
  return hipGetLastError();
}

hipError_t launch_sketch_reduce(const SketchPlan& p, int s, int n, const double* part,
                                double scale, double* B, int64_t ldb, hipStream_t st) {
  const size_t E = (size_t)p.it_total * p.jt_total * 256;
  const int blocks = (int)((E + 15) / 16);
  hipLaunchKernelGGL(k_sketch_reduce, dim3(blocks), dim3(256), 0, st, p.kblocks, p.it_total,
                     p.jt_total, s, n, part, scale, B, ldb);
  return hipGetLastError();
}

hipError_t launch_b_sketch(int IT, int JT, int NW, const BItem* items, int nitems,
                           const BProb* probs, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
#define TSQR_BSK(IT_, JT_, NW_)                                                          \
  if (IT == IT_ && JT == JT_ && NW == NW_) {                                             \
    hipLaunchKernelGGL((k_b_sketch<IT_, JT_, NW_>), dim3(nitems), dim3(NW_ * 64), 0, st, items, \
                       probs);                                                           \
    return hipGetLastError();                                                            \
  }
  TSQR_BSK(1, 1, 4) TSQR_BSK(1, 2, 4) TSQR_BSK(1, 4, 4) TSQR_BSK(1, 8, 4)
  TSQR_BSK(1, 1, 8) TSQR_BSK(1, 2, 8) TSQR_BSK(1, 4, 8) TSQR_BSK(1, 8, 8)
  TSQR_BSK(2, 8, 4) TSQR_BSK(2, 8, 8) TSQR_BSK(2, 4, 8) TSQR_BSK(2, 4, 4)
  TSQR_BSK(2, 2, 8) TSQR_BSK(2, 1, 8) TSQR_BSK(2, 2, 4) TSQR_BSK(2, 1, 4)
#undef TSQR_BSK
  return hipErrorInvalidValue;
}

hipError_t launch_b_sketch_reduce(const BItem* items, int nitems, const BProb* probs,
                                  hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_sketch_reduce, dim3(nitems), dim3(256), 0, st, items, probs);
  return hipGetLastError();
}

hipError_t launch_philox_words(int64_t count, const uint32_t* ctr, uint64_t seed, uint32_t* out,
                               hipStream_t st) {
  if (count <= 0) return hipSuccess;
  int blocks = (int)((count + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_philox_words, dim3(blocks), dim3(256), 0, st, count, ctr,
                     (uint32_t)seed, (uint32_t)(seed >> 32), out);
  return hipGetLastError();
}

hipError_t launch_sketch_normals(uint64_t seed, int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                                 double* Z, int64_t ldz, hipStream_t st) {
  const int64_t total = ni * nj;
  if (total <= 0) return hipSuccess;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_sketch_normals, dim3(blocks), dim3(256), 0, st, (uint32_t)seed,
                     (uint32_t)(seed >> 32), i0, ni, j0, nj, Z, ldz);
  return hipGetLastError();
}

}  // namespace tsqr
