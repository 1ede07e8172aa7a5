// Attainable-peak probes of the roofline: how many bytes per second the HBM delivers to a
// plain streaming kernel (read, write, copy) and how many flops per second the matrix
// cores sustain on independent MFMA chains (FP64, FP32, BF16 inputs).  They calibrate
// the rooflines against which the factorization's kernels are measured; none of them is
// part of the factorization.
#include "tsqr_device.hpp"
#include "tsqr_launch.hpp"

namespace tsqr {
namespace {

typedef double v2d_t __attribute__((ext_vector_type(2)));
typedef __bf16 v8bf_t __attribute__((ext_vector_type(8)));

constexpr int kProbeThreads = 256;

// kind 0: read  (sum of 16-byte words)
// kind 1: write (fill with a constant)
// kind 2: copy
// Thread t of the grid handles words t + k stride (stride = grid size), U of them per
// loop trip so that U loads are in flight per thread.  NT: nontemporal (streaming)
// stores.
template <int U, bool NT>
__global__ __launch_bounds__(kProbeThreads) void k_probe_stream(int kind,
                                                               const v2d_t* __restrict__ src,
                                                               v2d_t* __restrict__ dst,
                                                               int64_t words, double* sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (kind == 0) {
    v2d_t acc = {0.0, 0.0};
    for (; i + (U - 1) * stride < words; i += U * stride) {
      v2d_t v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = src[i + u * stride];
#pragma unroll
      for (int u = 0; u < U; ++u) acc += v[u];
    }
    for (; i < words; i += stride) acc += src[i];
    const double v = wave_sum(acc.x + acc.y);
    if (lane_id() == 0 && v == 12345.678) sink[0] = v;  // keeps the loads live
  } else if (kind == 1) {
    const v2d_t c = {1.0, 1.0};
    for (; i < words; i += stride) {
      if (NT)
        __builtin_nontemporal_store(c, dst + i);
      else
        dst[i] = c;
    }
  } else {
    for (; i + (U - 1) * stride < words; i += U * stride) {
      v2d_t v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = src[i + u * stride];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (NT)
          __builtin_nontemporal_store(v[u], dst + i + u * stride);
        else
          dst[i + u * stride] = v[u];
      }
    }
    for (; i < words; i += stride) dst[i] = src[i];
  }
}

// kind 0: FP64 16x16x4 (2048 flops), 1: FP32 16x16x4 (2048), 2: BF16 16x16x32 (16384),
// 3: BF16 32x32x16 (32768).  C independent accumulator chains per wavefront, `iters`
// steps of each.
// (the occupancy hint keeps the accumulators in VGPRs: without it the compiler held them
// in AGPRs and copied all of them out and back on every iteration, so the loop measured
// the copies, 51 TFLOP/s, rather than the matrix core)
// RND: the operands change at every step, to random doubles in [0.5, 1) (52 varying
// mantissa bits from a linear congruential sequence per lane), as the operands of the
// method's kernels do; the matrix core's sustained rate depends on its data.
template <int C, bool RND = false>
__global__ __launch_bounds__(kProbeThreads) __attribute__((amdgpu_waves_per_eu(2))) void
k_probe_mfma_f64(int64_t iters, double seed, double* sink) {
  v4d acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
  double a = seed + threadIdx.x, b = 1.0 / (1.0 + threadIdx.x);
  uint32_t h = 2654435761u * (threadIdx.x + 1u) + blockIdx.x;
  for (int64_t it = 0; it < iters; ++it) {
    if constexpr (RND) {
      h = h * 1664525u + 1013904223u;
      const uint32_t h2 = h * 22695477u + 1u;
      a = __builtin_bit_cast(double, 0x3FE0000000000000ull |
                                         ((unsigned long long)(h & 0xFFFFFu) << 32) | h2);
      b = __builtin_bit_cast(double, 0x3FE0000000000000ull |
                                         ((unsigned long long)(h2 & 0xFFFFFu) << 32) | h);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = mfma_f64(a, b, acc[c]);
  }
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < C; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == 12345.678) sink[0] = s;
}

template <int C>
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma_f32(int64_t iters, double seed,
                                                                 double* sink) {
  v4f acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
  const float a = (float)seed + threadIdx.x, b = 1.f / (1.f + threadIdx.x);
  for (int64_t it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < C; ++c)
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < C; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == 12345.678f) sink[0] = s;
}

template <int C>
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma_bf16(int64_t iters, double seed,
                                                                  double* sink) {
  v4f acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = v4f{0.f, 0.f, 0.f, 0.f};
  v8bf_t a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)((float)seed + (float)(threadIdx.x + e));
    b[e] = (__bf16)(1.f / (1.f + (float)(threadIdx.x + e)));
  }
  for (int64_t it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < C; ++c)
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < C; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (s == 12345.678f) sink[0] = s;
}

typedef float v16f_t __attribute__((ext_vector_type(16)));

template <int C>
__global__ __launch_bounds__(kProbeThreads) void k_probe_mfma_bf16_32(int64_t iters, double seed,
                                                                     double* sink) {
  v16f_t acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[c][e] = 0.f;
  v8bf_t a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)((float)seed + (float)(threadIdx.x + e));
    b[e] = (__bf16)(1.f / (1.f + (float)(threadIdx.x + e)));
  }
  for (int64_t it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < C; ++c)
      acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[c], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[c][e];
  if (s == 12345.678f) sink[0] = s;
}

template <int C>
hipError_t probe_mfma_t(int kind, int blocks, int64_t iters, double* sink, hipStream_t st) {
  if (kind == 0)
    hipLaunchKernelGGL(k_probe_mfma_f64<C>, dim3(blocks), dim3(kProbeThreads), 0, st, iters, 0.5,
                       sink);
  else if (kind == 1)
    hipLaunchKernelGGL(k_probe_mfma_f32<C>, dim3(blocks), dim3(kProbeThreads), 0, st, iters, 0.5,
                       sink);
  else if (kind == 2)
    hipLaunchKernelGGL(k_probe_mfma_bf16<C>, dim3(blocks), dim3(kProbeThreads), 0, st, iters,
                       0.5, sink);
  else if (kind == 4)
    hipLaunchKernelGGL((k_probe_mfma_f64<C, true>), dim3(blocks), dim3(kProbeThreads), 0, st,
                       iters, 0.5, sink);
  else
    hipLaunchKernelGGL(k_probe_mfma_bf16_32<C>, dim3(blocks), dim3(kProbeThreads), 0, st, iters,
                       0.5, sink);
  return hipGetLastError();
}

}  // namespace

// wgs_per_cu: workgroups of 256 threads per compute unit (1..64); unroll: 1, 2, 4 or 8
// words per thread per trip; nontemporal: streaming stores
hipError_t launch_probe_stream(int kind, const void* src, void* dst, size_t bytes,
                               int wgs_per_cu, int unroll, int nontemporal, double* sink,
                               hipStream_t st) {
  const int64_t words = (int64_t)(bytes / 16);
  const int64_t cap = (int64_t)device_cu_count() * wgs_per_cu;
  int64_t blocks = (words + kProbeThreads - 1) / kProbeThreads;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
#define TSQR_PS(U, NT)                                                                       \
  if (unroll == U && (nontemporal != 0) == NT) {                                             \
    hipLaunchKernelGGL((k_probe_stream<U, NT>), dim3((unsigned)blocks), dim3(kProbeThreads), 0, \
                       st, kind, (const v2d_t*)src, (v2d_t*)dst, words, sink);               \
    return hipGetLastError();                                                                \
  }
  TSQR_PS(1, false) TSQR_PS(2, false) TSQR_PS(4, false) TSQR_PS(8, false)
  TSQR_PS(1, true) TSQR_PS(2, true) TSQR_PS(4, true) TSQR_PS(8, true)
#undef TSQR_PS
  return hipErrorInvalidValue;
}

// waves_per_simd: 1, 2, 4 or 8 (workgroups of 4 wavefronts per CU); chains: 4, 8 or 16.
// The flops of one launch are returned in *flops.
hipError_t launch_probe_mfma(int kind, int waves_per_simd, int chains, int64_t iters,
                             double* sink, double* flops, hipStream_t st) {
  const int blocks = device_cu_count() * waves_per_simd;
  const double per = kind == 3 ? 32768.0 : (kind == 2 ? 16384.0 : 2048.0);
  *flops = (double)blocks * (kProbeThreads / kWave) * chains * (double)iters * per;
  if (chains == 4) return probe_mfma_t<4>(kind, blocks, iters, sink, st);
  if (chains == 8) return probe_mfma_t<8>(kind, blocks, iters, sink, st);
  if (chains == 16) return probe_mfma_t<16>(kind, blocks, iters, sink, st);
  return hipErrorInvalidValue;
}

}  // namespace tsqr
