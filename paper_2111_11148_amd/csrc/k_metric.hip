// Accuracy metrics of a computed factorization, the two quantities by which the paper
// judges its algorithms (Section 4.2): orthogonality ||Q^T Q - I||_F and the relative
// residual ||A - Q R||_F / ||A||_F.  Both are evaluated with double-double accumulation
// (error-free products by FMA and error-free sums), so that values near the FP64 unit
// roundoff are resolved: a plain FP64 dot product over m rows carries an error of about
// sqrt(m) u relative to the sum of |terms|, which at m = 2^20 is far above 1e-15.
//
// Summation order is fixed (per-thread loops, then fixed trees), so the results are
// bitwise reproducible.  Entry point: tsqr_metrics (tsqr_api.hip).
#include "tsqr_device.hpp"
#include "tsqr_launch.hpp"

// The error-free transformations below rely on every sum and product being rounded as
// written: no contraction of a product and a sum into one FMA.
#pragma clang fp contract(off)

namespace tsqr {
namespace {

constexpr int kMetThreads = 256;
constexpr int kMetChunk = 64;  // rows (or k indices) staged in LDS per step

// (hi, lo) += a * b: the product split exactly into p + pe (FMA), p added to hi with
// Knuth's two-sum, both rounding errors gathered into lo.
__device__ __forceinline__ void dd_fma(double& hi, double& lo, double a, double b) {
  const double p = a * b;
  const double pe = __builtin_fma(a, b, -p);
  const double s = hi + p;
  const double v = s - hi;
  const double e = (hi - (s - v)) + (p - v);
  hi = s;
  lo += e + pe;
}

// (hi, lo) += x
__device__ __forceinline__ void dd_add(double& hi, double& lo, double x) {
  const double s = hi + x;
  const double v = s - hi;
  const double e = (hi - (s - v)) + (x - v);
  hi = s;
  lo += e;
}

// (hi, lo) += (h2, l2)
__device__ __forceinline__ void dd_add_dd(double& hi, double& lo, double h2, double l2) {
  dd_add(hi, lo, h2);
  lo += l2;
}

// Tree sum of one (hi, lo) pair per thread over the workgroup, in a fixed order; the
// result is valid in thread 0.
__device__ void block_dd_sum(double& hi, double& lo) {
  __shared__ double sh[kMetThreads], sl[kMetThreads];
  const int t = threadIdx.x;
  sh[t] = hi;
  sl[t] = lo;
  __syncthreads();
  for (int w = kMetThreads / 2; w > 0; w >>= 1) {
    if (t < w) {
      double h = sh[t], l = sl[t];
      dd_add_dd(h, l, sh[t + w], sl[t + w]);
      sh[t] = h;
      sl[t] = l;
    }
    __syncthreads();
  }
  hi = sh[0];
  lo = sl[0];
  __syncthreads();
}

__device__ __forceinline__ void upper_tile(int t, int& a, int& b) {
  b = 0;
  while ((b + 1) * (b + 2) / 2 <= t) ++b;
  a = t - b * (b + 1) / 2;
}

// Gram entries of Q in double-double: workgroup (tile pair p, row block rb) sums
// Q(r, 16a + i) Q(r, 16b + j) over the rows r of block rb for the upper tile pair
// (a, b) = upper_tile(p); thread 16 i + j owns entry (i, j).  part[(p nrb + rb) 256 + t]
// receives (hi, lo).
__global__ __launch_bounds__(kMetThreads) void k_met_gram(int64_t m, int n,
                                                          const double* __restrict__ Q,
                                                          int64_t ldq, int64_t rows_per_block,
                                                          int nrb, double2* __restrict__ part) {
  const int p = blockIdx.x, rb = blockIdx.y;
  int a, b;
  upper_tile(p, a, b);
  __shared__ double sa[kMetChunk][17], sb[kMetChunk][17];
  const int t = threadIdx.x, i = t / 16, j = t % 16;
  const int64_t r0 = (int64_t)rb * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < m ? r0 + rows_per_block : m;
  double hi = 0.0, lo = 0.0;
  for (int64_t c = r0; c < r1; c += kMetChunk) {
    for (int e = t; e < kMetChunk * 16; e += kMetThreads) {
      const int rr = e % kMetChunk, cc = e / kMetChunk;
      const int64_t row = c + rr;
      const int ca = 16 * a + cc, cb = 16 * b + cc;
      sa[rr][cc] = (row < r1 && ca < n) ? Q[(int64_t)ca * ldq + row] : 0.0;
      sb[rr][cc] = (row < r1 && cb < n) ? Q[(int64_t)cb * ldq + row] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < kMetChunk; ++rr) dd_fma(hi, lo, sa[rr][i], sb[rr][j]);
    __syncthreads();
  }
  part[((size_t)p * nrb + rb) * kMetThreads + t] = make_double2(hi, lo);
}

// Per tile pair: each entry summed over the row blocks in order, the identity subtracted
// in double-double, then sum of w e^2 with weight w = 2 for entries off the diagonal of
// Q^T Q (their mirror image is not computed), 1 on it, 0 below the diagonal of a
// diagonal tile and outside n.  pair_sum[p] = (hi, lo).
__global__ __launch_bounds__(kMetThreads) void k_met_gram_fin(int n, int nrb,
                                                              const double2* __restrict__ part,
                                                              double2* __restrict__ pair_sum) {
  const int p = blockIdx.x;
  int a, b;
  upper_tile(p, a, b);
  const int t = threadIdx.x, i = t / 16, j = t % 16;
  const int ci = 16 * a + i, cj = 16 * b + j;
  double hi = 0.0, lo = 0.0;
  for (int rb = 0; rb < nrb; ++rb) {
    const double2 v = part[((size_t)p * nrb + rb) * kMetThreads + t];
    dd_add_dd(hi, lo, v.x, v.y);
  }
  if (ci == cj) dd_add(hi, lo, -1.0);
  const double e = hi + lo;
  double w = 0.0;
  if (ci < n && cj < n) w = ci < cj ? 2.0 : (ci == cj ? 1.0 : 0.0);
  double sh = 0.0, sl = 0.0;
  dd_fma(sh, sl, w * e, e);
  block_dd_sum(sh, sl);
  if (t == 0) pair_sum[p] = make_double2(sh, sl);
}

// out[0] = sqrt(sum over the tile pairs)
__global__ __launch_bounds__(kMetThreads) void k_met_gram_final(int npairs,
                                                                const double2* __restrict__ ps,
                                                                double* __restrict__ out) {
  double hi = 0.0, lo = 0.0;
  for (int p = threadIdx.x; p < npairs; p += kMetThreads) dd_add_dd(hi, lo, ps[p].x, ps[p].y);
  block_dd_sum(hi, lo);
  if (threadIdx.x == 0) out[0] = sqrt(hi + lo);
}

// Residual: thread = one row r, workgroup = 256 rows x one 16-column tile ct of A and R.
// e(r, c) = A(r, c) - sum_k Q(r, k) R(k, c) in double-double over every k < n (R as
// given), then sums of e^2 and of A(r, c)^2; part[(ct gridDim.x + bx)] = (num, den), each
// a (hi, lo) pair.
__global__ __launch_bounds__(kMetThreads) void k_met_res(int64_t m, int n,
                                                         const double* __restrict__ A,
                                                         int64_t lda,
                                                         const double* __restrict__ Q,
                                                         int64_t ldq,
                                                         const double* __restrict__ R,
                                                         int64_t ldr, double4* __restrict__ part) {
  const int ct = blockIdx.y;
  const int t = threadIdx.x;
  const int64_t row = (int64_t)blockIdx.x * kMetThreads + t;
  const bool rok = row < m;
  const int64_t rowc = rok ? row : 0;
  __shared__ double sr[kMetChunk][16];
  double eh[16], el[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int col = 16 * ct + c;
    eh[c] = (rok && col < n) ? A[(int64_t)col * lda + row] : 0.0;
    el[c] = 0.0;
  }
  for (int k0 = 0; k0 < n; k0 += kMetChunk) {
    for (int e = t; e < kMetChunk * 16; e += kMetThreads) {
      const int kk = e % kMetChunk, c = e / kMetChunk;
      const int k = k0 + kk, col = 16 * ct + c;
      sr[kk][c] = (k < n && col < n) ? R[(int64_t)col * ldr + k] : 0.0;
    }
    __syncthreads();
    const int kn = n - k0 < kMetChunk ? n - k0 : kMetChunk;
    for (int kk = 0; kk < kn; ++kk) {
      const double q = -Q[(int64_t)(k0 + kk) * ldq + rowc];
#pragma unroll
      for (int c = 0; c < 16; ++c) dd_fma(eh[c], el[c], q, sr[kk][c]);
    }
    __syncthreads();
  }
  double nh = 0.0, nl = 0.0, dh = 0.0, dl = 0.0;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const int col = 16 * ct + c;
    if (rok && col < n) {
      const double e = eh[c] + el[c];
      dd_fma(nh, nl, e, e);
      const double av = A[(int64_t)col * lda + row];
      dd_fma(dh, dl, av, av);
    }
  }
  block_dd_sum(nh, nl);
  block_dd_sum(dh, dl);
  if (t == 0) part[(size_t)ct * gridDim.x + blockIdx.x] = make_double4(nh, nl, dh, dl);
}

// out[1] = sqrt(num) / sqrt(den) over all partials
__global__ __launch_bounds__(kMetThreads) void k_met_res_final(int64_t nparts,
                                                               const double4* __restrict__ part,
                                                               double* __restrict__ out) {
  double nh = 0.0, nl = 0.0, dh = 0.0, dl = 0.0;
  for (int64_t p = threadIdx.x; p < nparts; p += kMetThreads) {
    dd_add_dd(nh, nl, part[p].x, part[p].y);
    dd_add_dd(dh, dl, part[p].z, part[p].w);
  }
  block_dd_sum(nh, nl);
  block_dd_sum(dh, dl);
  if (threadIdx.x == 0) out[1] = sqrt(nh + nl) / sqrt(dh + dl);
}

__global__ void k_met_nan(double* out) {
  if (threadIdx.x == 0) out[1] = __builtin_nan("");
}

struct MetPlan {
  int npairs, nrb;
  int64_t rows_per_block, res_blocks;
  int res_tiles;
  size_t gram_off, pair_off, res_off, total;
};

MetPlan plan_metrics(int64_t m, int n) {
  MetPlan p{};
  const int jt = (n + 15) / 16;
  p.npairs = jt * (jt + 1) / 2;
  // about 4096 workgroups for the Gram: enough row blocks to fill the GPU
  int64_t nrb = (4096 + p.npairs - 1) / p.npairs;
  const int64_t chunks = (m + kMetChunk - 1) / kMetChunk;
  if (nrb > chunks) nrb = chunks;
  if (nrb < 1) nrb = 1;
  const int64_t rpb_chunks = (chunks + nrb - 1) / nrb;
  p.rows_per_block = rpb_chunks * kMetChunk;
  p.nrb = (int)((m + p.rows_per_block - 1) / p.rows_per_block);
  p.res_blocks = (m + kMetThreads - 1) / kMetThreads;
  p.res_tiles = jt;
  size_t off = 0;
  p.gram_off = off;
  off += ((size_t)p.npairs * p.nrb * kMetThreads * sizeof(double2) + 255) & ~(size_t)255;
  p.pair_off = off;
  off += ((size_t)p.npairs * sizeof(double2) + 255) & ~(size_t)255;
  p.res_off = off;
  off += ((size_t)p.res_blocks * p.res_tiles * sizeof(double4) + 255) & ~(size_t)255;
  p.total = off;
  return p;
}

}  // namespace

size_t metrics_workspace_bytes(int64_t m, int n) { return plan_metrics(m, n).total; }

hipError_t launch_metrics(int64_t m, int n, const double* A, int64_t lda, const double* Q,
                          int64_t ldq, const double* R, int64_t ldr, double* out, void* work,
                          hipStream_t st) {
  const MetPlan p = plan_metrics(m, n);
  char* base = (char*)work;
  double2* gpart = (double2*)(base + p.gram_off);
  double2* psum = (double2*)(base + p.pair_off);
  double4* rpart = (double4*)(base + p.res_off);
  hipLaunchKernelGGL(k_met_gram, dim3(p.npairs, p.nrb), dim3(kMetThreads), 0, st, m, n, Q, ldq,
                     p.rows_per_block, p.nrb, gpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_met_gram_fin, dim3(p.npairs), dim3(kMetThreads), 0, st, n, p.nrb, gpart,
                     psum);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_met_gram_final, dim3(1), dim3(kMetThreads), 0, st, p.npairs, psum, out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (A && R) {
    hipLaunchKernelGGL(k_met_res, dim3((unsigned)p.res_blocks, p.res_tiles), dim3(kMetThreads), 0,
                       st, m, n, A, lda, Q, ldq, R, ldr, rpart);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_met_res_final, dim3(1), dim3(kMetThreads), 0, st,
                       (int64_t)p.res_blocks * p.res_tiles, rpart, out);
  } else {
    hipLaunchKernelGGL(k_met_nan, dim3(1), dim3(64), 0, st, out);
  }
  return hipGetLastError();
}

}  // namespace tsqr
