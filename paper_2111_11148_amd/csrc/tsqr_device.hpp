// Device-side building blocks shared by the HIP kernels of libtsqr (gfx950 / CDNA4).
//
//  * Philox4x32-10 counter-based generator and the Box-Muller map that define the
//    Gaussian sketch S (stream layout documented in include/tsqr.h);
//  * the FP64 MFMA 16x16x4 wrapper and its operand layouts;
//  * wavefront (64-lane) reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

namespace tsqr {

constexpr int kWave = 64;

// Upper-triangular tile numbering, column by column: tile t is (a, b) with
// t = b (b + 1) / 2 + a, a <= b.  UpperTile<t> evaluates the map at compile time (a
// template constant, so it is folded even where a loop over t would not be unrolled
// far enough for the optimiser to fold a constexpr call).
template <int T>
struct UpperTile {
  static constexpr int col() {
    int b = 0;
    while ((b + 1) * (b + 2) / 2 <= T) ++b;
    return b;
  }
  static constexpr int b = col();
  static constexpr int a = T - b * (b + 1) / 2;
};

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) double lds_f64;  // a double in LDS

// ---------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
//   (c0,c1,c2,c3) -> (hi(M1*c2)^c1^k0, lo(M1*c2), hi(M0*c0)^c3^k1, lo(M0*c0)),
// key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------------
struct U32x4 {
  uint32_t x, y, z, w;
};

// a ^ b ^ k in one instruction (v_bitop3_b32 with truth table 0x96 = three-input parity);
// k is uniform (the round key), so it is taken from a scalar register
__device__ __forceinline__ uint32_t xor3_key(uint32_t a, uint32_t b, uint32_t k) {
  uint32_t r;
  asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
  return r;
}

__device__ __forceinline__ U32x4 philox4x32_10(U32x4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round) {
      k0 += W0;
      k1 += W1;
    }
    // one 32 x 32 -> 64-bit product per multiplier (v_mad_u64_u32) gives both halves
    const uint64_t p0 = (uint64_t)M0 * c.x, p1 = (uint64_t)M1 * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = U32x4{xor3_key(hi1, c.y, k0), lo1, xor3_key(hi0, c.w, k1), lo0};
  }
  return c;
}

// Box-Muller on 24-bit uniforms, evaluated in single precision with the hardware
// transcendentals: u = ((wa>>8)+1) 2^-24 in (0,1], t = (wb>>8) 2^-24 in [0,1) are exact in
// FP32; v_log_f32 is log2, v_sin_f32 / v_cos_f32 take their argument in turns
// (sin(2 pi t)).  Returns (rad cos 2 pi t, rad sin 2 pi t).
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, float& z0, float& z1) {
  const float u = (float)((wa >> 8) + 1u) * 0x1p-24f;
  const float t = (float)(wb >> 8) * 0x1p-24f;
  // -2 ln u = -2 ln(2) log2(u)
  const float rad = __builtin_amdgcn_sqrtf(-1.3862943611198906f * __builtin_amdgcn_logf(u));
  z0 = rad * __builtin_amdgcn_cosf(t);
  z1 = rad * __builtin_amdgcn_sinf(t);
}

// The four N(0,1) entries Z(i, 4p..4p+3) of the sketch (one Philox call).
__device__ __forceinline__ void sketch_normals4(uint64_t p, uint32_t i, uint32_t k0, uint32_t k1,
                                                float z[4]) {
  const U32x4 w = philox4x32_10(U32x4{(uint32_t)p, (uint32_t)(p >> 32), i, 0u}, k0, k1);
  box_muller(w.x, w.y, z[0], z[1]);
  box_muller(w.z, w.w, z[2], z[3]);
}

// ---------------------------------------------------------------------------------
// V_MFMA_F64_16X16X4_F64: D(16x16) = A(16x4) B(4x16) + C.  Lane l (0..63) supplies
//   A[l%16][l/16] and B[l/16][l%16], and holds D[4*r + l/16][l%16] in register r = 0..3
//   (measured on gfx950; note the row interleave of the accumulator).
// ---------------------------------------------------------------------------------
__device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------------
// Wavefront reductions (64 lanes, butterfly; every lane gets the result).
// ---------------------------------------------------------------------------------
// DPP move of a double (two 32-bit halves) with a row-level control code
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the 64 lanes, the same (uniform) value in every lane: DPP within rows of 16
// lanes (swap pairs, swap halves of quads, rotate by 4 and by 8), then the four row sums
// read into scalars and added in a fixed order.  All lanes must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x124>(v);  // row_ror:4
  v += dpp_f64<0x128>(v);  // row_ror:8
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// sum over kb = k0, k0 + stride, ... < kblocks of part[kb E + e], in increasing kb, with
// eight loads in flight: the adds keep the order of the plain loop (so the result is the
// same), but the loads no longer wait for one another
__device__ __forceinline__ double strided_sum(const double* __restrict__ part, size_t E,
                                              size_t e, int k0, int stride, int kblocks) {
  double acc = 0.0;
  int kb = k0;
  for (; kb + 7 * stride < kblocks; kb += 8 * stride) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(size_t)(kb + u * stride) * E + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; kb < kblocks; kb += stride) acc += part[(size_t)kb * E + e];
  return acc;
}

// The same (wave-uniform) value read from the first active lane, so that the compiler
// keeps it in scalar registers: needed where it feeds an inline-assembly scalar operand in
// a kernel whose control flow hides that it is uniform.
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  return reinterpret_cast<T*>(uniform_i64(reinterpret_cast<int64_t>(p)));
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
// wavefront index inside the workgroup, as a uniform (scalar) value
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
}

}  // namespace tsqr
