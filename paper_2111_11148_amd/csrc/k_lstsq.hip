// Least squares min ||A x - b||_2 preconditioned by the sketch's R factor (paper Section
// 5.2): the kernels beyond the method's own, c = B^T b for B = A R0^{-1} and the three
// n x n triangular solves.
#include <hip/hip_runtime.h>

#include "tsqr_device.hpp"
#include "tsqr_launch.hpp"

namespace tsqr {

// c partials: workgroup kb sums rows [kb rpb, (kb + 1) rpb) of X^T b.  A wavefront takes
// 8 columns at a time (8 independent loads per row step), its lanes stride over the rows,
// and wave_sum reduces the lanes in a fixed order (deterministic).
constexpr int kGemvCols = 8;

__global__ __launch_bounds__(256) void k_gemv_t(int64_t m, int n, const double* __restrict__ X,
                                                int64_t ldx, const double* __restrict__ b,
                                                int64_t rows_per_block, double* __restrict__ part) {
  const int lane = lane_id(), wave = wave_id(), nw = blockDim.x / kWave;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(m, r0 + rows_per_block);
  for (int j0 = wave * kGemvCols; j0 < n; j0 += nw * kGemvCols) {
    double acc[kGemvCols];
#pragma unroll
    for (int u = 0; u < kGemvCols; ++u) acc[u] = 0.0;
    for (int64_t row = r0 + lane; row < r1; row += kWave) {
      const double bv = b[row];
#pragma unroll
      for (int u = 0; u < kGemvCols; ++u) {
        const int j = j0 + u < n ? j0 + u : n - 1;  // valid column; its sum is not stored
        acc[u] += X[(int64_t)j * ldx + row] * bv;
      }
    }
#pragma unroll
    for (int u = 0; u < kGemvCols; ++u) {
      const double t = wave_sum(acc[u]);
      if (lane == 0 && j0 + u < n) part[(size_t)blockIdx.x * n + j0 + u] = t;
    }
  }
}

// c(j) = sum over kb of part[kb][j]: workgroup j, thread t sums kb = t, t + 256, ... in
// increasing order, then the 256 sums are added in a fixed order (wave_sum within each
// wavefront, the four wavefront sums in order).  Each thread's loads are independent, so
// they are in flight together.
__global__ __launch_bounds__(256) void k_gemv_reduce(int kblocks, int n,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ c) {
  __shared__ double ws[4];
  const int j = blockIdx.x, t = threadIdx.x, lane = lane_id(), wave = wave_id();
  double acc = 0.0;
  for (int kb = t; kb < kblocks; kb += 256) acc += part[(size_t)kb * n + j];
  acc = wave_sum(acc);
  if (lane == 0) ws[wave] = acc;
  __syncthreads();
  if (t == 0) c[j] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// One wavefront, the vector in LDS (a single wavefront's LDS accesses are in order, so no
// barrier is needed), the triangular factor's next column loaded while the current step
// runs: U^T z = c (z_i = (c_i - sum_{k<i} U(k,i) z_k) / U(i,i), column i of U read
// contiguously, wave_sum for the dot product), U y = z and R0 x = y (column-oriented back
// substitution: y_i = z_i / U(i,i), then z_k -= U(k,i) y_i for k < i).  RL: rows per lane
// (n <= 64 RL).  Skipped (x = NaN) when *info is set.
template <int RL>
__global__ __launch_bounds__(64) void k_lsq_solve(int n, const double* __restrict__ U,
                                                  int64_t ldu, const double* __restrict__ R0,
                                                  int64_t ldr, const double* __restrict__ c,
                                                  double* __restrict__ x,
                                                  const int* __restrict__ info) {
  extern __shared__ double v[];  // n doubles
  const int lane = threadIdx.x;
  if (*info != 0) {
    for (int i = lane; i < n; i += kWave) x[i] = NAN;
    return;
  }
  for (int i = lane; i < n; i += kWave) v[i] = c[i];
  __builtin_amdgcn_wave_barrier();
  // column j of T, rows lane + 64 r (row 0 stands in past n: a valid address)
  auto load_col = [&](const double* T, int64_t ldt, int j, double (&col)[RL]) {
    const int jc = j < n ? j : n - 1;
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int k = lane + kWave * r;
      col[r] = T[(int64_t)jc * ldt + (k < n ? k : 0)];
    }
  };
  double cur[RL], nxt[RL];
  // forward: U^T z = c, z overwrites v
  load_col(U, ldu, 0, cur);
  for (int i = 0; i < n; ++i) {
    load_col(U, ldu, i + 1, nxt);
    const double uii = U[(int64_t)i * ldu + i];
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < RL; ++r) {
      const int k = lane + kWave * r;
      acc += (k < i) ? cur[r] * v[k < n ? k : 0] : 0.0;
    }
    acc = wave_sum(acc);
    if (lane == 0) v[i] = (v[i] - acc) / uii;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int r = 0; r < RL; ++r) cur[r] = nxt[r];
  }
  // back: U y = z, then R0 x = y, y and x overwrite v
  for (int pass = 0; pass < 2; ++pass) {
    const double* T = pass == 0 ? U : R0;
    const int64_t ldt = pass == 0 ? ldu : ldr;
    load_col(T, ldt, n - 1, cur);
    for (int i = n - 1; i >= 0; --i) {
      load_col(T, ldt, i > 0 ? i - 1 : 0, nxt);
      const double tii = T[(int64_t)i * ldt + i];
      const double yi = v[i] / tii;  // every lane reads v[i] and divides alike
      __builtin_amdgcn_wave_barrier();
      if (lane == 0) v[i] = yi;
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int k = lane + kWave * r;
        if (k < i) v[k] -= cur[r] * yi;
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int r = 0; r < RL; ++r) cur[r] = nxt[r];
    }
  }
  for (int i = lane; i < n; i += kWave) x[i] = v[i];
}

int64_t gemv_rows_per_block(int64_t m) {
  const int64_t target = (int64_t)device_cu_count() * 2;
  int64_t rpb = (m + target - 1) / target;
  rpb = ((rpb + 63) / 64) * 64;
  return rpb < 64 ? 64 : rpb;
}

hipError_t launch_gemv_t(int64_t m, int n, const double* X, int64_t ldx, const double* b,
                         double* part, double* c, hipStream_t st) {
  const int64_t rpb = gemv_rows_per_block(m);
  const int kblocks = (int)((m + rpb - 1) / rpb);
  hipLaunchKernelGGL(k_gemv_t, dim3(kblocks), dim3(256), 0, st, m, n, X, ldx, b, rpb, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gemv_reduce, dim3(n), dim3(256), 0, st, kblocks, n, part, c);
  return hipGetLastError();
}

size_t gemv_part_doubles(int64_t m, int n) {
  const int64_t rpb = gemv_rows_per_block(m);
  return (size_t)((m + rpb - 1) / rpb) * (size_t)n;
}

hipError_t launch_lsq_solve(int n, const double* U, int64_t ldu, const double* R0, int64_t ldr,
                            const double* c, double* x, const int* info, hipStream_t st) {
  const size_t sh = (size_t)n * sizeof(double);
#define TSQR_LSQ(RL_)                                                                          \
  if (n <= 64 * RL_) {                                                                         \
    hipLaunchKernelGGL(k_lsq_solve<RL_>, dim3(1), dim3(kWave), sh, st, n, U, ldu, R0, ldr, c, x, \
                       info);                                                                  \
    return hipGetLastError();                                                                  \
  }
  TSQR_LSQ(1) TSQR_LSQ(2) TSQR_LSQ(4) TSQR_LSQ(8) TSQR_LSQ(16)
#undef TSQR_LSQ
  return hipErrorInvalidValue;
}

}  // namespace tsqr
