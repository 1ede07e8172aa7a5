// Batched randomized XR-preconditioned CholeskyQR: many independent problems of uneven
// sizes factored together (each problem is the method of paper Algorithm rQR- or
// rLU-CholeskyQR with the Gaussian sketch of Section 2.3 and one more CholeskyQR pass).
//
// Every phase of the chain is one launch per width class over a work list that holds the
// workgroups of all problems of that class, so the machine is filled by the batch rather
// than by any single problem.  A plan (built once on the host) groups the problems into
// classes, sizes each problem's split-K blocking and triangular-solve grid, lays out the
// workspace and uploads the problem descriptors and work lists into it.  Running a plan
// only enqueues kernels: no allocation, no copy and no host synchronisation, so the whole
// batch can be captured into one HIP graph and replayed.
#include <algorithm>
#include <cmath>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "tsqr_launch.hpp"

namespace tsqr {
namespace {

size_t align256b(size_t b) { return (b + 255) & ~(size_t)255; }

int pow2_ceil(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

size_t trsm_tiles_doubles(int jt) {
  return (size_t)(jt * (jt - 1) / 2 + 2 * jt) * 256 + (size_t)(jt + 1) / 2 + 1;
}

// Width class of a problem: everything that selects a kernel instantiation.
struct ClassKey {
  int jt;               // 16-column tiles of the panel (power of two)
  int sk_it, sk_nw;     // sketch: i-tiles per wave, waves per workgroup
  int sk_jt;            // sketch: column tiles per workgroup
  int qr_rpl, qr_cpw;   // register factorization of the sketch
  int po_rpl, po_cpw;   // register Cholesky
  bool operator<(const ClassKey& o) const {
    return std::tie(jt, sk_it, sk_nw, sk_jt, qr_rpl, qr_cpw, po_rpl, po_cpw) <
           std::tie(o.jt, o.sk_it, o.sk_nw, o.sk_jt, o.qr_rpl, o.qr_cpw, o.po_rpl, o.po_cpw);
  }
};

struct Launch {
  int phase;  // see run()
  ClassKey key;
  size_t first;  // offset into the item array
  int count;
};

}  // namespace
}  // namespace tsqr

struct tsqr_batch {
  int variant = 0;
  int precision = 0;  // TSQR_BATCH_FP64, or TSQR_LOWP_FP32 / TSQR_LOWP_BF16 for the sketch
  int64_t count = 0;
  size_t probs_off = 0, items_off = 0;
  tsqr::BProb* probs_dev = nullptr;
  tsqr::BItem* items_dev = nullptr;
  std::vector<tsqr::Launch> launches;
  // the persistent schedule: task queue, queue head and abort flag, dynamic LDS
  int4* ptasks_dev = nullptr;
  int nptasks = 0;
  int* pctl_dev = nullptr;
  size_t plds = 0;
};

namespace tsqr {
namespace {

enum Phase {
  kSetInfo, kSketch, kSketchReduce, kFactor, kPrep0, kTrsmA, kGram1, kGramReduce1, kPotrf1,
  kTrmm10, kPrep1, kTrsm1, kGram2, kGramReduce2, kPotrf2, kTrmmR, kPrep2, kTrsm2, kPoison,
  kNumPhases
};

// Blocking of a plan: rows per split-K workgroup of the sketch and of the Gram kernels,
// 16-row tiles per triangular-solve workgroup.  The defaults let one workgroup stream a
// few thousand rows (enough to amortise its partial-sum write) while the batch still
// spreads over the whole GPU; tsqr_batched_autotune measures the alternatives.
constexpr tsqr_batch_tuning kDefaultTuning = {2048, 2048, 64};
// smallest blockings the autotuner tries (they bound the workspace)
constexpr int64_t kMinRows = 1024;
constexpr int kMinTiles = 32;

struct Layout {
  size_t total = 0;
  std::vector<size_t> off;  // per problem: start of its buffers
};

size_t problem_doubles(int64_t m, int n, int s, const tsqr_batch_tuning& t) {
  const int jt = pow2_ceil((n + 15) / 16);
  const int it_total = (s + 15) / 16, jt_total = (n + 15) / 16;
  const int sk_k = (int)((m + t.sketch_rows - 1) / t.sketch_rows);
  const int gr_k = (int)((m + t.gram_rows - 1) / t.gram_rows);
  const size_t sk_part = (size_t)sk_k * it_total * jt_total * 256;
  const size_t gr_part = (size_t)gr_k * (jt_total * (jt_total + 1) / 2) * 256;
  const size_t nn = (size_t)n * n;
  size_t d = 0;
  d += align256b((size_t)s * n * 8) / 8;             // B
  d += 5 * (align256b(nn * 8) / 8);                  // R0 R1 R2 R10 W
  d += align256b(trsm_tiles_doubles(jt) * 8) / 8;    // P
  d += align256b(std::max(sk_part, gr_part) * 8) / 8;
  return d;
}

// Codes in the numbering of tsqr_batched_create (count is argument 3, problems 4).
int validate(int64_t count, const tsqr_problem* pr) {
  if (count < 1) return -3;
  if (!pr) return -4;
  for (int64_t i = 0; i < count; ++i) {
    const tsqr_problem& q = pr[i];
    if (q.n < 1 || q.n > 128 || q.m < q.n || q.s < q.n || q.s > 512 || !q.A || q.lda < q.m ||
        !q.Q || q.ldq < q.m || (q.R && q.ldr < q.n))
      return -4;
    // the register-resident factorization of the sketch holds s x n in one workgroup:
    // 8 rows and 8 columns per lane do not fit, so s <= 256 when n > 64
    if (q.n > 64 && q.s > 256) return -4;
  }
  return 0;
}

// Header of the workspace: problem descriptors, the per-phase work items, the persistent
// task queue, its head and abort flag, and each problem's dependency counters.
constexpr int kCntStride = 16;  // ints per problem (kPsSlots used)
static_assert(kPsSlots <= kCntStride, "counter slots");

size_t header_bytes(int64_t count, size_t nitems, size_t ntasks) {
  return align256b((size_t)count * sizeof(BProb)) + align256b(nitems * sizeof(BItem)) +
         align256b(ntasks * sizeof(int4)) + 256 + align256b((size_t)count * kCntStride * 4);
}

// Sketch i-groups of the persistent schedule (16 wavefronts of one 16-row tile each).
int persist_igroups(int s) { return ((s + 15) / 16 + 15) / 16; }

}  // namespace
}  // namespace tsqr

using namespace tsqr;

extern "C" {

size_t tsqr_batched_workspace_bytes(int64_t count, const tsqr_problem* problems) {
  if (validate(count, problems) != 0) return 0;
  // sized for the smallest blockings, so that every tuning fits
  const tsqr_batch_tuning t{kMinRows, kMinRows, kMinTiles};
  size_t items = 0, tasks = 0, bufs = 0;
  for (int64_t i = 0; i < count; ++i) {
    const tsqr_problem& q = problems[i];
    const int n = (int)q.n, s = (int)q.s;
    const int it_total = (s + 15) / 16, jt_total = (n + 15) / 16;
    const int jt = pow2_ceil(jt_total);
    const int sk_jt = std::min(jt, 8);
    const int sk_it = it_total >= 16 ? 2 : 1;
    const int waves = (it_total + sk_it - 1) / sk_it;
    const int sk_nw = waves >= 8 ? 8 : 4;
    const int ig = (it_total + sk_nw * sk_it - 1) / (sk_nw * sk_it);
    const int jg = (jt_total + sk_jt - 1) / sk_jt;
    const int sk_k = (int)((q.m + t.sketch_rows - 1) / t.sketch_rows);
    const int gr_k = (int)((q.m + t.gram_rows - 1) / t.gram_rows);
    const int64_t ntiles = (q.m + 15) / 16;
    const int twg = (int)std::min<int64_t>(256, (ntiles + t.trsm_tiles - 1) / t.trsm_tiles);
    const size_t e_sk = (size_t)it_total * jt_total * 256, e_gr = (size_t)(jt_total * (jt_total + 1) / 2) * 256;
    items += 1 + (size_t)sk_k * ig * jg + (e_sk + 15) / 16 + 1 + 3 * jt + 3 * twg +
             2 * ((size_t)gr_k + (e_gr + 15) / 16) + 2 + 2 * (size_t)jt_total * jt_total + 4;
    tasks += (size_t)sk_k * persist_igroups(s) * ((jt_total + 3) / 4) + 3 * (size_t)twg +
             2 * (size_t)gr_k;
    bufs += align256b(problem_doubles(q.m, n, s, t) * 8);
  }
  return header_bytes(count, items, tasks) + bufs;
}

int tsqr_batched_create(int variant, int precision, int64_t count, const tsqr_problem* problems,
                        void* work, size_t work_bytes, int* d_info,
                        const tsqr_batch_tuning* tuning, tsqr_batch** out) {
  if (variant != TSQR_VARIANT_RQR && variant != TSQR_VARIANT_RLU) return -1;
  if (precision != TSQR_BATCH_FP64 && precision != TSQR_LOWP_FP32 && precision != TSQR_LOWP_BF16)
    return -2;
  const int v = validate(count, problems);
  if (v) return v;
  if (!work) return -5;
  if (!d_info) return -7;
  const tsqr_batch_tuning t = tuning ? *tuning : kDefaultTuning;
  if (t.sketch_rows < kMinRows || t.sketch_rows % 64 || t.gram_rows < kMinRows ||
      t.gram_rows % 64 || t.trsm_tiles < kMinTiles)
    return -8;
  if (!out) return -9;
  *out = nullptr;
  const size_t need = tsqr_batched_workspace_bytes(count, problems);
  if (work_bytes < need) return TSQR_ERR_WORKSPACE;

  std::vector<BProb> probs((size_t)count);
  std::vector<ClassKey> keys((size_t)count);
  // per phase, per class: the items
  std::map<ClassKey, std::vector<BItem>> items[kNumPhases];
  size_t nitems = 0;
  // buffers after the header; the header size depends on the item count, so lay buffers
  // out relative to a base fixed after counting
  std::vector<size_t> buf_off((size_t)count);
  size_t bufs = 0;
  for (int64_t i = 0; i < count; ++i) {
    const tsqr_problem& q = problems[i];
    BProb& p = probs[(size_t)i];
    const int n = (int)q.n, s = (int)q.s;
    p.A = q.A;
    p.Q = q.Q;
    p.R = q.R;
    p.m = q.m;
    p.lda = q.lda;
    p.ldq = q.ldq;
    p.ldr = q.R ? q.ldr : n;
    p.n = n;
    p.s = s;
    p.k0 = (uint32_t)q.seed;
    p.k1 = (uint32_t)(q.seed >> 32);
    p.scale = 1.0 / std::sqrt((double)s);
    p.info = d_info + i;
    const int it_total = (s + 15) / 16, jt_total = (n + 15) / 16;
    ClassKey k{};
    k.jt = pow2_ceil(jt_total);
    k.sk_jt = std::min(k.jt, 8);
    k.sk_it = it_total >= 16 ? 2 : 1;
    const int waves = (it_total + k.sk_it - 1) / k.sk_it;
    k.sk_nw = waves >= 8 ? 8 : 4;
    k.qr_rpl = pow2_ceil((s + 63) / 64);
    k.qr_cpw = pow2_ceil((n + 15) / 16);
    k.po_rpl = pow2_ceil((n + 63) / 64);
    k.po_cpw = pow2_ceil((n + 15) / 16);
    keys[(size_t)i] = k;
    p.sk_it = it_total;
    p.sk_jt = jt_total;
    p.sk_rpb = t.sketch_rows;
    p.sk_kblocks = (int)((q.m + t.sketch_rows - 1) / t.sketch_rows);
    p.gr_rpb = t.gram_rows;
    p.gr_kblocks = (int)((q.m + t.gram_rows - 1) / t.gram_rows);
    p.gr_ntiles = jt_total * (jt_total + 1) / 2;
    const int64_t ntiles = (q.m + 15) / 16;
    p.trsm_wgs = (int)std::min<int64_t>(256, (ntiles + t.trsm_tiles - 1) / t.trsm_tiles);
    p.poison_wgs = 4;
    p.jt = k.jt;
    p.qr_rpl = k.qr_rpl;
    p.qr_cpw = k.qr_cpw;
    p.po_rpl = k.po_rpl;
    p.po_cpw = k.po_cpw;
    p.p_igroups = persist_igroups(s);
    p.p_jgroups = precision == TSQR_BATCH_FP64 ? 1 : (jt_total + 3) / 4;
    p.p_nsk = p.sk_kblocks * p.p_igroups * p.p_jgroups;
    p.p_ntrsm = p.trsm_wgs;
    buf_off[(size_t)i] = bufs;
    bufs += align256b(problem_doubles(q.m, n, s, t) * 8);

    const int pid = (int)i;
    auto add = [&](int phase, int x, int y, int z) {
      items[phase][k].push_back(BItem{pid, x, y, z});
      ++nitems;
    };
    add(kSetInfo, 0, 0, 0);
    const int ig = (it_total + k.sk_nw * k.sk_it - 1) / (k.sk_nw * k.sk_it);
    const int jg = (jt_total + k.sk_jt - 1) / k.sk_jt;
    for (int kb = 0; kb < p.sk_kblocks; ++kb)
      for (int a = 0; a < ig; ++a)
        for (int b = 0; b < jg; ++b) add(kSketch, kb, a, b);
    const size_t e_sk = (size_t)it_total * jt_total * 256;
    for (size_t g = 0; g < (e_sk + 15) / 16; ++g) add(kSketchReduce, (int)g, 0, 0);
    add(kFactor, 0, 0, 0);
    for (int b = 0; b < k.jt; ++b) {
      add(kPrep0, b, 0, 0);
      add(kPrep1, b, 0, 0);
      add(kPrep2, b, 0, 0);
    }
    for (int w = 0; w < p.trsm_wgs; ++w) {
      add(kTrsmA, w, 0, 0);
      add(kTrsm1, w, 0, 0);
      add(kTrsm2, w, 0, 0);
    }
    for (int kb = 0; kb < p.gr_kblocks; ++kb) {
      add(kGram1, kb, 0, 0);
      add(kGram2, kb, 0, 0);
    }
    const size_t e_gr = (size_t)p.gr_ntiles * 256;
    for (size_t g = 0; g < (e_gr + 15) / 16; ++g) {
      add(kGramReduce1, (int)g, 0, 0);
      add(kGramReduce2, (int)g, 0, 0);
    }
    add(kPotrf1, 0, 0, 0);
    add(kPotrf2, 0, 0, 0);
    for (int a = 0; a < jt_total; ++a)
      for (int b = 0; b < jt_total; ++b) {
        add(kTrmm10, a, b, 0);
        add(kTrmmR, a, b, 0);
      }
    for (int w = 0; w < p.poison_wgs; ++w) add(kPoison, w, 0, 0);
  }

  // the persistent queue: phase by phase, and within a phase the problems with the most
  // work first (their tasks are the longest), each problem's tasks together
  std::vector<int> order((size_t)count);
  for (int64_t i = 0; i < count; ++i) order[(size_t)i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const BProb& pa = probs[(size_t)a];
    const BProb& pb = probs[(size_t)b];
    return (double)pa.m * pa.n * (2.0 * pa.s + 5.0 * pa.n) >
           (double)pb.m * pb.n * (2.0 * pb.s + 5.0 * pb.n);
  });
  std::vector<int4> ptasks;
  for (int kind = 0; kind < 6; ++kind) {
    // queue order of the kinds: sketch, solve by R0, Gram 1, solve by R1, Gram 2, solve by R2
    const int k = kind == 0 ? 0 : kind == 1 ? 1 : kind == 2 ? 4 : kind == 3 ? 2 : kind == 4 ? 5 : 3;
    for (int pid : order) {
      const BProb& p = probs[(size_t)pid];
      if (k == 0) {
        for (int bx = 0; bx < p.sk_kblocks; ++bx)
          for (int y = 0; y < p.p_igroups * p.p_jgroups; ++y)
            ptasks.push_back(int4{0, pid, bx, y});
      } else if (k <= 3) {
        for (int w = 0; w < p.p_ntrsm; ++w) ptasks.push_back(int4{k, pid, w, 0});
      } else {
        for (int bx = 0; bx < p.gr_kblocks; ++bx) ptasks.push_back(int4{k, pid, bx, 0});
      }
    }
  }

  // workspace: [descriptors | work items | persistent tasks | head, abort | counters |
  //             per-problem buffers]
  char* base = (char*)work;
  const size_t probs_bytes = align256b((size_t)count * sizeof(BProb));
  const size_t items_bytes = align256b(nitems * sizeof(BItem));
  const size_t tasks_bytes = align256b(ptasks.size() * sizeof(int4));
  const size_t cnt_bytes = align256b((size_t)count * kCntStride * 4);
  char* tasks_base = base + probs_bytes + items_bytes;
  int* ctl_base = (int*)(tasks_base + tasks_bytes);
  int* cnt_base = ctl_base + 64;
  char* bufbase = (char*)cnt_base + cnt_bytes;
  if (probs_bytes + items_bytes + tasks_bytes + 256 + cnt_bytes + bufs > work_bytes)
    return TSQR_ERR_WORKSPACE;
  for (int64_t i = 0; i < count; ++i) {
    BProb& p = probs[(size_t)i];
    p.cnt = cnt_base + (size_t)i * kCntStride;
    const int n = p.n, s = p.s;
    const size_t nn = (size_t)n * n;
    char* c = bufbase + buf_off[(size_t)i];
    p.B = (double*)c;
    c += align256b((size_t)s * n * 8);
    p.R0 = (double*)c;
    c += align256b(nn * 8);
    p.R1 = (double*)c;
    c += align256b(nn * 8);
    p.R2 = (double*)c;
    c += align256b(nn * 8);
    p.R10 = (double*)c;
    c += align256b(nn * 8);
    p.W = (double*)c;
    c += align256b(nn * 8);
    p.P = (double*)c;
    c += align256b(trsm_tiles_doubles(pow2_ceil((n + 15) / 16)) * 8);
    p.part = (double*)c;
  }

  tsqr_batch* plan = new (std::nothrow) tsqr_batch;
  if (!plan) return TSQR_ERR_HIP;
  plan->variant = variant;
  plan->precision = precision;
  plan->count = count;
  plan->probs_dev = (BProb*)base;
  plan->items_dev = (BItem*)(base + probs_bytes);
  plan->ptasks_dev = (int4*)tasks_base;
  plan->nptasks = (int)ptasks.size();
  plan->pctl_dev = ctl_base;
  {
    int max_jt = 1;
    for (const BProb& p : probs) max_jt = std::max(max_jt, p.jt);
    plan->plds = persistent_lds_bytes(max_jt, 0, precision);
  }
  std::vector<BItem> all;
  all.reserve(nitems);
  for (int ph = 0; ph < kNumPhases; ++ph)
    for (auto& kv : items[ph]) {
      plan->launches.push_back(Launch{ph, kv.first, all.size(), (int)kv.second.size()});
      all.insert(all.end(), kv.second.begin(), kv.second.end());
    }
  if (hipMemcpy(plan->probs_dev, probs.data(), (size_t)count * sizeof(BProb),
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(plan->items_dev, all.data(), all.size() * sizeof(BItem), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(plan->ptasks_dev, ptasks.data(), ptasks.size() * sizeof(int4),
                hipMemcpyHostToDevice) != hipSuccess) {
    delete plan;
    return TSQR_ERR_HIP;
  }
  *out = plan;
  return TSQR_OK;
}

int tsqr_batched_run(tsqr_batch* plan, void* stream) {
  if (!plan) return -1;
  hipStream_t st = (hipStream_t)stream;
  const BProb* P = plan->probs_dev;
  for (const Launch& L : plan->launches) {
    const BItem* it = plan->items_dev + L.first;
    const ClassKey& k = L.key;
    hipError_t e = hipSuccess;
    switch (L.phase) {
      case kSetInfo: e = launch_b_set_info(it, L.count, P, st); break;
      case kSketch:
        e = plan->precision == TSQR_BATCH_FP64
                ? launch_b_sketch(k.sk_it, k.sk_jt, k.sk_nw, it, L.count, P, st)
                : launch_b_sketch_lowp(plan->precision, k.sk_it, k.sk_jt, k.sk_nw, it, L.count,
                                       P, st);
        break;
      case kSketchReduce: e = launch_b_sketch_reduce(it, L.count, P, st); break;
      case kFactor: e = launch_b_factor(plan->variant, k.qr_rpl, k.qr_cpw, it, L.count, P, st); break;
      case kPrep0: e = launch_b_trsm_prep(0, it, L.count, P, st); break;
      case kTrsmA: e = launch_b_trsm(k.jt, 0, it, L.count, P, st); break;
      case kGram1:
      case kGram2: e = launch_b_gram(k.jt, it, L.count, P, st); break;
      case kGramReduce1:
      case kGramReduce2: e = launch_b_gram_reduce(it, L.count, P, st); break;
      case kPotrf1: e = launch_b_potrf(k.po_rpl, k.po_cpw, 1, 2, it, L.count, P, st); break;
      case kPotrf2: e = launch_b_potrf(k.po_rpl, k.po_cpw, 2, 3, it, L.count, P, st); break;
      case kTrmm10: e = launch_b_trmm(0, it, L.count, P, st); break;
      case kPrep1: e = launch_b_trsm_prep(1, it, L.count, P, st); break;
      case kTrsm1: e = launch_b_trsm(k.jt, 1, it, L.count, P, st); break;
      case kTrmmR: e = launch_b_trmm(1, it, L.count, P, st); break;
      case kPrep2: e = launch_b_trsm_prep(2, it, L.count, P, st); break;
      case kTrsm2: e = launch_b_trsm(k.jt, 1, it, L.count, P, st); break;
      case kPoison: e = launch_b_poison(it, L.count, P, st); break;
      default: e = hipErrorInvalidValue;
    }
    if (e != hipSuccess) return TSQR_ERR_HIP;
  }
  return TSQR_OK;
}

}  // extern "C"

namespace tsqr {
namespace {

// Coordinate search over the sketch blocking, the Gram blocking and the solve grid of a
// plan, each from four candidates, timing the phase-by-phase schedule or the persistent
// launch (which prefers coarser tasks: its per-task publish and the solve's operand
// staging are paid once per task).
int autotune(bool persistent, int variant, int precision, int64_t count,
             const tsqr_problem* problems, void* work, size_t work_bytes, int* d_info,
             void* stream, tsqr_batch_tuning* best, double* best_ms) {
  if (!best) return -9;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return TSQR_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);  // best effort on the error path
    return TSQR_ERR_HIP;
  }
  auto run = [&](tsqr_batch* plan) {
    return persistent ? tsqr_batched_run_persistent(plan, st) : tsqr_batched_run(plan, st);
  };
  // time of one run of the batch planned with `t` (warm-up run, then the mean of two)
  auto measure = [&](const tsqr_batch_tuning& t, double* ms) -> int {
    tsqr_batch* plan = nullptr;
    int rc = tsqr_batched_create(variant, precision, count, problems, work, work_bytes, d_info, &t,
                                 &plan);
    if (rc) return rc;
    rc = run(plan);
    if (!rc && hipEventRecord(e0, st) != hipSuccess) rc = TSQR_ERR_HIP;
    for (int r = 0; r < 2 && !rc; ++r) rc = run(plan);
    if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = TSQR_ERR_HIP;
    if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = TSQR_ERR_HIP;
    float f = 0.f;
    if (!rc && hipEventElapsedTime(&f, e0, e1) != hipSuccess) rc = TSQR_ERR_HIP;
    tsqr_batched_destroy(plan);
    *ms = f / 2.0;
    return rc;
  };
  tsqr_batch_tuning cur = persistent ? tsqr_batch_tuning{4096, 4096, 128} : kDefaultTuning;
  double cur_ms = 0.0;
  int rc = measure(cur, &cur_ms);
  const int64_t rows_phase[] = {1024, 2048, 4096, 8192};
  const int64_t rows_persist[] = {2048, 4096, 8192, 16384};
  const int tiles_phase[] = {32, 64, 128, 256};
  const int tiles_persist[] = {64, 128, 256, 512};
  const int64_t* rows = persistent ? rows_persist : rows_phase;
  const int* tiles = persistent ? tiles_persist : tiles_phase;
  for (int dim = 0; dim < 3 && !rc; ++dim)
    for (int c = 0; c < 4 && !rc; ++c) {
      tsqr_batch_tuning t = cur;
      if (dim == 0) t.sketch_rows = rows[c];
      if (dim == 1) t.gram_rows = rows[c];
      if (dim == 2) t.trsm_tiles = tiles[c];
      if (t.sketch_rows == cur.sketch_rows && t.gram_rows == cur.gram_rows &&
          t.trsm_tiles == cur.trsm_tiles)
        continue;
      double ms = 0.0;
      rc = measure(t, &ms);
      if (!rc && ms < cur_ms) {
        cur = t;
        cur_ms = ms;
      }
    }
  const hipError_t d0 = hipEventDestroy(e0), d1 = hipEventDestroy(e1);
  if (rc) return rc;
  if (d0 != hipSuccess || d1 != hipSuccess) return TSQR_ERR_HIP;
  *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return TSQR_OK;
}

}  // namespace
}  // namespace tsqr

extern "C" {

int tsqr_batched_autotune(int variant, int precision, int64_t count,
                          const tsqr_problem* problems, void* work, size_t work_bytes, int* d_info,
                          void* stream, tsqr_batch_tuning* best, double* best_ms) {
  return autotune(false, variant, precision, count, problems, work, work_bytes, d_info, stream,
                  best, best_ms);
}

int tsqr_batched_autotune_persistent(int variant, int precision, int64_t count,
                                     const tsqr_problem* problems, void* work, size_t work_bytes,
                                     int* d_info, void* stream, tsqr_batch_tuning* best,
                                     double* best_ms) {
  return autotune(true, variant, precision, count, problems, work, work_bytes, d_info, stream,
                  best, best_ms);
}

int tsqr_batched_run_persistent(tsqr_batch* plan, void* stream) {
  return tsqr_batched_run_persistent_timed(plan, nullptr, stream);
}

int tsqr_batched_run_persistent_timed(tsqr_batch* plan, unsigned long long* d_stats,
                                      void* stream) {
  if (!plan) return -1;
  if (launch_b_persistent(plan->variant, plan->precision, plan->probs_dev, (int)plan->count,
                          plan->ptasks_dev, plan->nptasks, plan->pctl_dev, plan->plds, d_stats,
                          (hipStream_t)stream) != hipSuccess)
    return TSQR_ERR_HIP;
  return TSQR_OK;
}

int tsqr_batched_tasks(const tsqr_batch* plan) { return plan ? plan->nptasks : 0; }

int tsqr_batched_launches(const tsqr_batch* plan) {
  return plan ? (int)plan->launches.size() : 0;
}

void tsqr_batched_destroy(tsqr_batch* plan) { delete plan; }

}  // extern "C"
