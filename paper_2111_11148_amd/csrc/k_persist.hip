// One persistent launch for a whole batch of factorizations.
//
// Every workgroup (16 wavefronts, one per compute unit) takes tasks from a queue that the
// plan lays out phase by phase: all sketch tasks, then the solves by R0, the first Gram
// matrices, the solves by R1, the second Gram matrices and the solves by R2, each phase
// over every problem.  Per-problem counters in device memory replace the kernel
// boundaries of the phase-by-phase schedule: a task first waits until the step it reads
// is complete for its own problem only, so the phases of different problems overlap.  The
// workgroup that completes the last split-K task of a problem's sketch or Gram matrix
// finishes that step itself: the fixed-order reduction of the partial sums, the small
// factorization (Householder QR or partial-pivot LU of the sketch, Cholesky of the Gram
// matrix), the R product and the preparation of the next solve's operand tiles.
//
// Ordering across workgroups (possibly on different XCDs with separate L2 caches): a
// finished task publishes with an agent-scope release fence before its counter increment;
// a waiting workgroup polls the counter with relaxed atomic loads and issues an
// agent-scope acquire fence once it is satisfied.  The queue only hands out a task after
// every task it depends on has been handed out to a running workgroup, so every wait ends;
// a wait is still bounded, and a workgroup that gives up raises an abort flag on which
// every workgroup exits (all problems then report info = 9000).
#include "tsqr_device.hpp"
#include "tsqr_launch.hpp"

namespace tsqr {

constexpr int kPersistThreads = kSmallThreads;  // 16 wavefronts
static_assert(kPersistThreads == 1024, "the bodies below assume 16 wavefronts");
constexpr uint32_t kSpinLimit = 1u << 25;  // polls of about 0.1 us: a few seconds

__device__ __forceinline__ int load_relaxed(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0: wait until *p >= target (then acquire), or until the abort flag is raised or
// the poll limit is reached (then false).
__device__ bool wait_at_least(const int* p, int target, const int* abort_flag) {
  for (uint32_t i = 0;; ++i) {
    if (load_relaxed(p) >= target) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      return true;
    }
    if (load_relaxed(abort_flag) || i >= kSpinLimit) return false;
    __builtin_amdgcn_s_sleep(2);
  }
}

// A copy of a small descriptor held in scalar registers: every 32-bit word is read from
// lane 0.  The task taken from the queue (its index comes through LDS) is made uniform this
// way, so that the problem descriptor it names is read with scalar loads, as the bodies
// expect of the sizes, strides, pointers and keys they pass to inline assembly as scalar
// operands.
template <class T>
__device__ __forceinline__ T uniform_copy(const T& v) {
  static_assert(sizeof(T) % 4 == 0, "whole words");
  T out;
  const int* src = reinterpret_cast<const int*>(&v);
  int* dst = reinterpret_cast<int*>(&out);
#pragma unroll
  for (int w = 0; w < (int)(sizeof(T) / 4); ++w) dst[w] = __builtin_amdgcn_readfirstlane(src[w]);
  return out;
}

// Runtime class value -> compile-time constant (powers of two up to 8).
template <int V>
struct IC {
  static constexpr int value = V;
};
template <class F>
__device__ __forceinline__ void with_pow2(int v, F&& f) {
  switch (v) {
    case 1: f(IC<1>{}); break;
    case 2: f(IC<2>{}); break;
    case 4: f(IC<4>{}); break;
    default: f(IC<8>{}); break;
  }
}

// Fixed-order reduction of split-K partials (tile-native FP64, kblocks of E entries) by the
// whole workgroup: entry e is summed over the row blocks in increasing order.
template <class Put>
__device__ __forceinline__ void reduce_partials(int kblocks, size_t E,
                                                const double* __restrict__ part, Put put) {
  for (size_t e = threadIdx.x; e < E; e += blockDim.x) {
    put(e, strided_sum(part, E, e, 0, 1, kblocks));
  }
}

// C = A B for upper triangular n x n A, B (C upper, strict lower part zeroed); entry
// (i, j) sums k = i..j in increasing order.  C must not overlap A or B.
__device__ __forceinline__ void block_trmm_upper(int n, const double* __restrict__ A,
                                                 const double* __restrict__ B,
                                                 double* __restrict__ C, int64_t ldc) {
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e % n, j = e / n;
    double acc = 0.0;
    for (int k = i; k <= j; ++k) acc += A[(int64_t)k * n + i] * B[(int64_t)j * n + k];
    C[(int64_t)j * ldc + i] = i <= j ? acc : 0.0;
  }
}

// Operand tiles of the solve by T (n x n, ld n) into p.P, one block column after another.
__device__ __forceinline__ void prepare_solve(const BProb& p, const double* T) {
  for (int b = 0; b < p.jt; ++b) {
    trsm_prep_body(p.n, p.jt, T, p.n, p.P, b);
    __syncthreads();
  }
}

// Finisher of a problem's sketch: B = scale * (sum of the partials), R0 from B, operand
// tiles of the solve by R0.
__device__ void finish_sketch(const BProb& p, int variant, double* lds) {
  const size_t E = (size_t)p.sk_it * p.sk_jt * 256;
  reduce_partials(p.sk_kblocks, E, p.part, [&](size_t e, double t) {
    const int tile = (int)(e / 256), lane = (int)((e / 4) % 64), r = (int)(e % 4);
    const int itg = tile / p.sk_jt, jtg = tile % p.sk_jt;
    const int i = 16 * itg + 4 * r + (lane >> 4), c = 16 * jtg + (lane & 15);
    if (i < p.s && c < p.n) p.B[(int64_t)c * p.s + i] = p.scale * t;
  });
  __syncthreads();
  with_pow2(p.qr_rpl, [&](auto rpl) {
    with_pow2(p.qr_cpw, [&](auto cpw) {
      constexpr int RPL = decltype(rpl)::value, CPW = decltype(cpw)::value;
      // the register factorization holds at most 32 entries per lane (s <= 256 at n > 64)
      if constexpr (RPL * CPW <= 32) {
        if (variant == TSQR_VARIANT_RLU)
          getrf_reg_body<RPL, CPW, true>(p.s, p.n, p.B, p.s, p.R0, p.n, p.info, lds);
        else
          geqrf_reg_body<RPL, CPW, true>(p.s, p.n, p.B, p.s, p.R0, p.n, p.info, lds);
      }
    });
  });
  __syncthreads();
  prepare_solve(p, p.R0);
}

// Finisher of a problem's Gram matrix g (1 or 2): W = sum of the partials, Rg = chol(W),
// the R product (R10 = R1 R0, or R = R2 R10) and the operand tiles of the solve by Rg.
__device__ void finish_gram(const BProb& p, int g) {
  const size_t E = (size_t)p.gr_ntiles * 256;
  reduce_partials(p.gr_kblocks, E, p.part, [&](size_t e, double t) {
    const int tile = (int)(e / 256), lane = (int)((e / 4) % 64), r = (int)(e % 4);
    const int a = tri_a(tile), b = tri_b(tile);
    const int i = 16 * a + 4 * r + (lane >> 4), j = 16 * b + (lane & 15);
    if (i < p.n && j < p.n) {
      p.W[(int64_t)j * p.n + i] = t;
      p.W[(int64_t)i * p.n + j] = t;
    }
  });
  __syncthreads();
  double* Rg = g == 1 ? p.R1 : p.R2;
  with_pow2(p.po_rpl, [&](auto rpl) {
    with_pow2(p.po_cpw, [&](auto cpw) {
      constexpr int RPL = decltype(rpl)::value, CPW = decltype(cpw)::value;
      // n <= 128: two rows per lane at most
      if constexpr (RPL <= 2) potrf_reg_body<RPL, CPW>(p.n, p.W, p.n, Rg, p.n, g + 1, p.info, 0.0);
    });
  });
  __syncthreads();
  if (g == 1)
    block_trmm_upper(p.n, p.R1, p.R0, p.R10, p.n);
  else if (p.R)
    block_trmm_upper(p.n, p.R2, p.R10, p.R, p.ldr);
  prepare_solve(p, Rg);
}

// The problem broke down somewhere (info != 0): Q and R become NaN.
__device__ void poison_problem(const BProb& p) {
  const double nan = __builtin_nan("");
  for (int64_t e = threadIdx.x; e < p.m * p.n; e += blockDim.x)
    p.Q[(e / p.m) * p.ldq + e % p.m] = nan;
  if (p.R)
    for (int e = threadIdx.x; e < p.n * p.n; e += blockDim.x)
      p.R[(int64_t)(e / p.n) * p.ldr + e % p.n] = nan;
}

// Every task body is a function of its own, not inlined into the scheduler loop: the
// register allocator then sees one body at a time (inlined, all of them share one
// allocation and spill).  Arguments arrive in vector registers, so each entry reads its
// descriptor pointer and indices back from lane 0 to keep them scalar.
template <int PREC, int JT>
__device__ __attribute__((noinline)) void run_sketch(const BProb* pin, int bx, int y) {
  extern __shared__ double psm[];
  const BProb& p = *uniform_ptr(pin);
  bx = __builtin_amdgcn_readfirstlane(bx);
  y = __builtin_amdgcn_readfirstlane(y);
  const int by = y % p.p_igroups, bz = y / p.p_igroups;
  const uint32_t k0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)p.k0);
  const uint32_t k1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)p.k1);
  if constexpr (PREC == TSQR_BATCH_FP64) {
    sketch_f64_body<1, JT, 16, true>(p.m, p.n, p.A, p.lda, k0, k1, p.sk_rpb, p.sk_it, p.sk_jt,
                                     p.part, bx, by, bz, psm);
  } else {
    // at most 4 column tiles: the FP32 accumulators and their FP64 sums for 8 tiles would
    // not fit the registers of a 16-wavefront workgroup
    constexpr int JL = JT < 4 ? JT : 4;
    sketch_lowp_body<PREC, 1, JL, 16, true>(p.m, p.n, p.A, p.lda, k0, k1, p.sk_rpb, p.sk_it,
                                            p.sk_jt, p.part, bx, by, bz, psm);
  }
}

template <int JT>
__device__ __attribute__((noinline)) void run_solve(const BProb* pin, int kind, int wg) {
  const BProb& p = *uniform_ptr(pin);
  kind = __builtin_amdgcn_readfirstlane(kind);
  wg = __builtin_amdgcn_readfirstlane(wg);
  const double* Y = kind == 1 ? p.A : p.Q;
  const int64_t ldy = kind == 1 ? p.lda : p.ldq;
  trsm_mfma_body<JT, true>(p.m, p.n, Y, ldy, p.P, p.Q, p.ldq, wg, p.p_ntrsm);
}

template <int JT>
__device__ __attribute__((noinline)) void run_gram(const BProb* pin, int bx) {
  extern __shared__ double psm[];
  const BProb& p = *uniform_ptr(pin);
  bx = __builtin_amdgcn_readfirstlane(bx);
  gram_f64_body<JT, 16, 1, false, true>(p.m, p.n, p.Q, p.ldq, p.gr_rpb, p.gr_ntiles, p.part, bx,
                                        0, psm);
}

__device__ __attribute__((noinline)) void run_finish(const BProb* pin, int kind, int variant) {
  extern __shared__ double psm[];
  const BProb& p = *uniform_ptr(pin);
  kind = __builtin_amdgcn_readfirstlane(kind);
  variant = __builtin_amdgcn_readfirstlane(variant);
  if (kind == 0)
    finish_sketch(p, variant, psm);
  else if (kind >= 4)
    finish_gram(p, kind - 3);
  else if (kind == 3 && load_relaxed(p.info) != 0)
    poison_problem(p);
}

// Task kinds: 0 sketch (x row block, y i-group); 1, 2, 3 the solves by R0, R1, R2 (x the
// task's index among the solve's tasks); 4, 5 the Gram matrices 1, 2 (x row block).
// stats (optional, measurement): per task kind k, accumulated wall-clock ticks (100 MHz)
// of waiting at [3k], of the body at [3k+1] and of the finishing step at [3k+2].
template <int PREC>
__global__ __launch_bounds__(kPersistThreads, 1) void k_b_persistent(
    int variant, const BProb* __restrict__ probs, int nprobs, const int4* __restrict__ tasks,
    int ntasks, int* __restrict__ ctl, unsigned long long* __restrict__ stats) {
  extern __shared__ double psm[];  // the bodies' working LDS (the solve's tiles alias it)
  __shared__ int s_task, s_go, s_last;
  int* head = ctl;
  const int* abort_flag = ctl + 1;
  for (;;) {
    if (threadIdx.x == 0) {
      int t = atomicAdd(head, 1);
      if (load_relaxed(abort_flag)) t = ntasks;
      s_task = t;
    }
    __syncthreads();
    // uniform (scalar) task index: the task and problem descriptors are then scalar loads,
    // as the bodies expect of their sizes, strides and keys
    const int t = __builtin_amdgcn_readfirstlane(s_task);
    if (t >= ntasks) break;
    const int4 tk = uniform_copy(tasks[t]);
    const int kind = tk.x;
    const BProb& p = probs[tk.y];
    // the step this task reads must be complete for its problem
    uint64_t t0 = 0, t1 = 0, t2 = 0;
    if (threadIdx.x == 0) {
      if (stats) t0 = __builtin_amdgcn_s_memrealtime();
      bool ok = true;
      if (kind >= 1 && kind <= 3)
        ok = wait_at_least(p.cnt + (kind == 1 ? kPsR0 : kind == 2 ? kPsR1 : kPsR2), 1,
                           abort_flag);
      else if (kind >= 4)
        ok = wait_at_least(p.cnt + (kind == 4 ? kPsTrsm0 : kPsTrsm1), p.p_ntrsm, abort_flag);
      if (!ok) __hip_atomic_store(ctl + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_go = ok;
      if (stats) t1 = __builtin_amdgcn_s_memrealtime();
    }
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(s_go)) {
      for (int i = threadIdx.x; i < nprobs; i += blockDim.x) atomicCAS(probs[i].info, 0, 9000);
      break;
    }
    int slot, expected;
    if (kind == 0) {
      with_pow2(p.jt, [&](auto jt) { run_sketch<PREC, decltype(jt)::value>(&p, tk.z, tk.w); });
      slot = kPsSketch;
      expected = p.p_nsk;
    } else if (kind <= 3) {
      with_pow2(p.jt, [&](auto jt) { run_solve<decltype(jt)::value>(&p, kind, tk.z); });
      slot = kind == 1 ? kPsTrsm0 : kind == 2 ? kPsTrsm1 : kPsTrsm2;
      expected = p.p_ntrsm;
    } else {
      with_pow2(p.jt, [&](auto jt) { run_gram<decltype(jt)::value>(&p, tk.z); });
      slot = kind == 4 ? kPsGram1 : kPsGram2;
      expected = p.gr_kblocks;
    }
    // publish; the workgroup that completes the step finishes it
    __syncthreads();
    if (threadIdx.x == 0) {
      if (stats) t2 = __builtin_amdgcn_s_memrealtime();
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const int old = atomicAdd(p.cnt + slot, 1);
      s_last = old + 1 == expected;
      if (s_last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_last)) {
      run_finish(&p, kind, variant);
      const int ready = kind == 0 ? kPsR0 : kind == 4 ? kPsR1 : kind == 5 ? kPsR2 : -1;
      __syncthreads();
      if (ready >= 0 && threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(p.cnt + ready, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
    if (stats && threadIdx.x == 0) {
      const uint64_t t3 = __builtin_amdgcn_s_memrealtime();
      atomicAdd(stats + 3 * kind, (unsigned long long)(t1 - t0));
      atomicAdd(stats + 3 * kind + 1, (unsigned long long)(t2 - t1));
      atomicAdd(stats + 3 * kind + 2, (unsigned long long)(t3 - t2));
    }
  }
}

// Before each run: the queue head, the abort flag, every problem's counters and info.
__global__ void k_b_persistent_clear(const BProb* __restrict__ probs, int nprobs,
                                     int* __restrict__ ctl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 2) ctl[i] = 0;
  if (i < nprobs) {
    for (int k = 0; k < kPsSlots; ++k) probs[i].cnt[k] = 0;
    *probs[i].info = 0;
  }
}

size_t persistent_lds_bytes(int max_jt, int max_rpl_cpw, int precision) {
  size_t b = 0;
  auto upd = [&](size_t x) { b = x > b ? x : b; };
  for (int jt = 1; jt <= max_jt; jt <<= 1) {
    upd((size_t)(jt * (jt - 1) / 2 + 2 * jt) * 256 * sizeof(double));  // solve tiles
    upd((size_t)2 * 32 * (jt * 16 + 1) * sizeof(double));               // sketch / Gram
  }
  if (precision == TSQR_LOWP_FP32 || precision == TSQR_LOWP_BF16)
    for (int jt = 1; jt <= max_jt; jt <<= 1)  // the low-precision sketch's staging planes
      upd((size_t)jt * 16 * (precision == TSQR_LOWP_FP32 ? 65 * 4 : 72 * 6));
  upd((size_t)(2 * 64 * 8 + 16 * 8) * sizeof(double));                 // register factor
  (void)max_rpl_cpw;
  return b;
}

hipError_t launch_b_persistent(int variant, int precision, const BProb* probs, int nprobs,
                               const int4* tasks, int ntasks, int* ctl, size_t lds_bytes,
                               unsigned long long* stats, hipStream_t st) {
  hipLaunchKernelGGL(k_b_persistent_clear, dim3((nprobs + 255) / 256), dim3(256), 0, st, probs,
                     nprobs, ctl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid(device_cu_count()), block(kPersistThreads);
  if (precision == TSQR_BATCH_FP64)
    hipLaunchKernelGGL(k_b_persistent<TSQR_BATCH_FP64>, grid, block, lds_bytes, st, variant,
                       probs, nprobs, tasks, ntasks, ctl, stats);
  else if (precision == TSQR_LOWP_FP32)
    hipLaunchKernelGGL(k_b_persistent<TSQR_LOWP_FP32>, grid, block, lds_bytes, st, variant,
                       probs, nprobs, tasks, ntasks, ctl, stats);
  else
    hipLaunchKernelGGL(k_b_persistent<TSQR_LOWP_BF16>, grid, block, lds_bytes, st, variant,
                       probs, nprobs, tasks, ntasks, ctl, stats);
  return hipGetLastError();
}

}  // namespace tsqr
