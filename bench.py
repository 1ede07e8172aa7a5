#!/usr/bin/env python3
"""Throughput of randomized XR-preconditioned CholeskyQR on one MI355X.

One step = one whole factorization (sketch B = S A, R0 from the sketch, A1 = A R0^{-1},
Gram, Cholesky, Q1 = A1 R1^{-1}, the extra CholeskyQR pass and R = R2 R1 R0) of the
tall128 workload: m = 2^20, n = 128, s = 256, FP64, singular values log-spaced from 1 to
1e-14, rQR variant.  Inputs are resident in HBM before timing starts; workspace and
outputs are preallocated, so the timed region allocates nothing.

Printed: one JSON line with the throughput (GFLOP/s of the algorithmic flop count), the
roofline of the dominant kernel (average duration from HIP events recorded on the
library's stream around that kernel only, during the timed steps; the per-phase breakdown
comes from separate steps with events around every launch), the CPU oracle timed on a
bounded sample, and
the mixed-precision comparison: time to ||Q^T Q - I||_F <= 1e-12 on the mixed256 workload
(m = 2^20, n = 256, s = 512, kappa in {1e4, 1e8, 1e12}) for FP64 and for the FP32 / BF16
mixed variant, and the batched workload (512 uneven problems, one HIP graph per batch,
problems/s against a per-problem loop).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 (vector = matrix)
PEAK_HBM_GBS = 8000.0
METRIC = "tall-skinny QR GFLOP/s + roofline %, m=2^20 n=128; mixed vs FP64 at ortho≤1e-12"

# Kernel sources whose counter readings profiles/traffic_*.json refer to.
KERNEL_SOURCES = {
    "sketch": ["paper_2111_11148_amd/csrc/k_sketch.hip", "paper_2111_11148_amd/csrc/tsqr_device.hpp"],
    "trsm_r0": ["paper_2111_11148_amd/csrc/k_tall.hip", "paper_2111_11148_amd/csrc/tsqr_device.hpp"],
    "gram1": ["paper_2111_11148_amd/csrc/k_tall.hip", "paper_2111_11148_amd/csrc/tsqr_device.hpp"],
}


def flops(m: int, n: int, s: int, variant: str, extra_pass: bool) -> dict:
    """Algorithmic flop counts per phase (multiply-add = 2 flops)."""
    f = {
        "sketch": 2.0 * s * m * n,                     # B = S A
        "sketch_factor": (2.0 * n * n * (s - n / 3.0)) if variant == "rqr"
        else (1.0 * n * n * (s - n / 3.0)),            # Householder QR or LU of B
        "trsm": 1.0 * m * n * n,                       # one X = Y T^{-1}
        "gram": 1.0 * m * n * (n + 1),                 # upper triangle of X^T X
        "potrf": n ** 3 / 3.0,
        "trmm": n ** 3 / 3.0,
    }
    passes = 2 if extra_pass else 1
    total = (f["sketch"] + f["sketch_factor"] + (1 + passes) * f["trsm"] + passes * f["gram"]
             + passes * f["potrf"] + passes * f["trmm"])
    f["total"] = total
    return f


def source_hash(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, or None when absent or
    taken on a different version of the kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha") != source_hash(KERNEL_SOURCES[kernel]):
        return None
    return t.get("bytes_per_launch")


def gpu_metrics(A, Q, R):
    """Orthogonality and residual with blocked FP64 products on the device."""
    import torch

    m, n = A.shape
    G = None
    num = den = None
    Rc = R.contiguous()
    for r0 in range(0, m, 4096):
        q = Q[r0:r0 + 4096].contiguous()
        g = q.t().contiguous() @ q
        G = g if G is None else G + g
        a = A[r0:r0 + 4096]
        e = a - q @ Rc
        num = (e * e).sum() if num is None else num + (e * e).sum()
        den = (a * a).sum() if den is None else den + (a * a).sum()
    G -= torch.eye(n, dtype=G.dtype, device=G.device)
    return float(torch.linalg.matrix_norm(G)), float(torch.sqrt(num) / torch.sqrt(den))


def cached_matrix(cache_dir, name, m, n, kappa, seed):
    """The seeded test matrix, generated on the host (kept under cache_dir if given)."""
    import numpy as np

    from inputs import gen_matrix

    cache = None
    if cache_dir:
        os.makedirs(cache_dir, exist_ok=True)
        cache = os.path.join(cache_dir, f"A_{name}_{seed}.npy")
        if os.path.exists(cache):
            return np.load(cache, mmap_mode="r")
    t0 = time.perf_counter()
    A_h = gen_matrix(m, n, kappa, seed)
    print(f"# generated A ({m}x{n}, kappa={kappa:g}) in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    if cache:
        np.save(cache, np.asfortranarray(A_h))
    return A_h


def timed(fn, steps: int, warmup: int) -> float:
    """Average wall time per call in ms, device synchronised on both sides."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def phases_of(fn) -> dict:
    """Per-phase device time (ms) of one call, from the library's HIP events."""
    import torch

    import paper_2111_11148_amd as tsqr

    torch.cuda.synchronize()
    tsqr.profile_start()
    fn()
    torch.cuda.synchronize()
    out = {}
    for name, ms in tsqr.profile_stop():
        out[name] = round(out.get(name, 0.0) + ms, 4)
    return out


def mixed_comparison(args, kappas):
    """Time to an orthonormal Q (||Q^T Q - I||_F <= 1e-12) on the mixed256 workload:
    the FP64 method with one extra pass against the mixed variant with FP32 and with BF16
    inputs (automatic FP64 passes), same matrix, same GPU, each timed on its own."""
    import numpy as np
    import torch

    import paper_2111_11148_amd as tsqr
    from inputs import WORKLOADS

    wl = WORKLOADS["mixed256"]
    m, n, s, seed = wl.m, wl.n, wl.s, wl.sketch_seed
    F = flops(m, n, s, "rqr", True)["total"]
    Q = tsqr.colmajor(m, n)
    R = tsqr.colmajor(n, n)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    work64 = tsqr.alloc_workspace(m, n, s)
    out = []
    for kappa in kappas:
        j = list(wl.kappas).index(kappa)
        A_h = cached_matrix(args.cache_dir, wl.name, m, n, kappa, wl.gen_seeds[j])
        A = tsqr.to_device_colmajor(np.asarray(A_h))
        del A_h
        row = {"kappa": kappa}

        def fp64():
            tsqr.rxr_cholqr(A, s, seed, Q=Q, R=R, workspace=work64, info=info)

        ms = timed(fp64, args.mixed_steps, 2)
        ortho, res = gpu_metrics(A, Q, R)
        row["fp64"] = {"ms": round(ms, 4), "gflops": round(F / ms / 1e6, 2), "ortho": ortho,
                       "residual": res, "info": int(info.item()), "phases_ms": phases_of(fp64)}
        for name, lowp in (("fp32", tsqr.FP32), ("bf16", tsqr.BF16)):
            ws = torch.empty(tsqr.mixed_workspace_bytes(m, n, s, lowp), dtype=torch.uint8,
                             device="cuda")
            npass = []

            def mixed():
                npass.append(tsqr.rxr_cholqr_mixed(A, s, seed, lowp, Q=Q, R=R, workspace=ws,
                                                   info=info)[3])

            ms_m = timed(mixed, args.mixed_steps, 2)
            o_m, r_m = gpu_metrics(A, Q, R)
            ok = o_m <= 1e-12 and row["fp64"]["ortho"] <= 1e-12 and int(info.item()) == 0
            ph = phases_of(mixed)
            row[name] = {"ms": round(ms_m, 4), "gflops_equiv": round(F / ms_m / 1e6, 2),
                         "fp64_passes": npass[-1], "lowp_stage": "apply_lowp" in ph,
                         "ortho": o_m, "residual": r_m, "info": int(info.item()),
                         "speedup_vs_fp64": round(ms / ms_m, 3) if ok else None,
                         "phases_ms": ph}
            del ws
        out.append(row)
        print(f"# mixed kappa={kappa:g}: fp64 {row['fp64']['ms']:.3f} ms, fp32 "
              f"{row['fp32']['ms']:.3f} ms ({row['fp32']['fp64_passes']} passes), bf16 "
              f"{row['bf16']['ms']:.3f} ms ({row['bf16']['fp64_passes']} passes)",
              file=sys.stderr, flush=True)
        del A
        torch.cuda.empty_cache()
    return {"workload": f"{wl.name} (m={m}, n={n}, s={s}, rqr)", "flops_per_step": F,
            "target_ortho": 1e-12, "results": out}


def paper_shaped_comparison(args):
    """The paper's own strong-scaling problem (Table "scalability1": m = 1e7, n = 100,
    kappa = 1e5, l = 2n, rQR-CholeskyQR with row extraction as printed, CholeskyQR2 and
    sCholeskyQR3) on one GPU.  A (8 GB) is built on the device as U diag(sigma) V^T from
    seeded N(0,1) matrices orthonormalised by torch's QR (the construction of Section 4.1);
    it is timing input only and never meets the oracle."""
    import torch

    import paper_2111_11148_amd as tsqr

    m, n, s, kappa, seed = 10_000_000, 100, 200, 1e5, 11109
    gen = torch.Generator(device="cuda")
    gen.manual_seed(211109)
    G = torch.randn(m, n, generator=gen, dtype=torch.float64, device="cuda")
    U, _ = torch.linalg.qr(G)
    del G
    V, _ = torch.linalg.qr(torch.randn(n, n, generator=gen, dtype=torch.float64, device="cuda"))
    sig = kappa ** (-torch.arange(n, dtype=torch.float64, device="cuda") / (n - 1))
    A = tsqr.colmajor(m, n)
    A.copy_((U * sig) @ V.t())
    del U
    torch.cuda.empty_cache()
    Q, R = tsqr.colmajor(m, n), tsqr.colmajor(n, n)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    work = tsqr.alloc_workspace(m, n, s)
    cwork = torch.empty(tsqr.cholqr_workspace_bytes(m, n), dtype=torch.uint8, device="cuda")
    methods = {
        "rqr_rows": lambda: tsqr.rxr_cholqr(A, s, seed, extra_pass=False, Q=Q, R=R,
                                            workspace=work, info=info, sketch="rows"),
        "rqr_rows_plus_pass": lambda: tsqr.rxr_cholqr(A, s, seed, Q=Q, R=R, workspace=work,
                                                      info=info, sketch="rows"),
        "rqr_gaussian_plus_pass": lambda: tsqr.rxr_cholqr(A, s, seed, Q=Q, R=R, workspace=work,
                                                          info=info),
        "cholqr2": lambda: tsqr.cholqr(A, tsqr.CHOLQR2, Q=Q, R=R, workspace=cwork, info=info),
        "scholqr3": lambda: tsqr.cholqr(A, tsqr.SCHOLQR3, -1.0, Q=Q, R=R, workspace=cwork,
                                        info=info),
    }
    paper_s = {"rqr_rows": (1.8643, 0.052), "cholqr2": (2.3181, 0.0631),
               "scholqr3": (3.6855, 0.0958)}  # (8 processes, 512 processes), seconds
    out = {}
    for name, fn in methods.items():
        ms = timed(fn, args.baseline_steps, 1)
        code = int(info.item())
        o, r = gpu_metrics(A, Q, R) if code == 0 else (None, None)
        row = {"ms": round(ms, 3), "info": code, "ortho": o, "residual": r}
        if name in paper_s:
            row["paper_s_8_and_512_processes"] = paper_s[name]
            row["speedup_vs_paper_512_processes"] = round(paper_s[name][1] * 1e3 / ms, 2)
        out[name] = row
        print(f"# paper shape {name}: {ms:.3f} ms (info {code})", file=sys.stderr, flush=True)
    del A, Q, R, work, cwork
    torch.cuda.empty_cache()
    return {"workload": f"Table scalability1 shape (m={m}, n={n}, l={s}, kappa={kappa:g})",
            "results": out,
            "paper": "rQR-CholeskyQR (row extraction, no extra pass), CholeskyQR2 and "
                     "sCholeskyQR3 on 8-512 MPI processes of 32-core Xeon nodes"}


def baselines_comparison(args, kappas):
    """The paper's comparison (Section 4.3) on the benchmark's shape (m=2^20, n=128,
    s=256): rQR-CholeskyQR with the row-extraction sketch (the paper's experiments; as
    printed, and with the extra pass), with the Gaussian sketch (+1 pass, the headline
    method), CholeskyQR2 and sCholeskyQR3 (suggested shift), each timed on its own on the
    same matrix, with accuracy and breakdown codes."""
    import numpy as np
    import torch

    import paper_2111_11148_amd as tsqr

    m, n, s, seed = 1 << 20, 128, 256, 11108
    Q = tsqr.colmajor(m, n)
    R = tsqr.colmajor(n, n)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    work = tsqr.alloc_workspace(m, n, s)
    cwork = torch.empty(tsqr.cholqr_workspace_bytes(m, n), dtype=torch.uint8, device="cuda")
    out = []
    for j, kappa in enumerate(kappas):
        A_h = cached_matrix(args.cache_dir, f"baselines_{kappa:g}", m, n, kappa, 211108 + j)
        A = tsqr.to_device_colmajor(np.asarray(A_h))
        del A_h
        methods = {
            "rqr_rows": lambda: tsqr.rxr_cholqr(A, s, seed, extra_pass=False, Q=Q, R=R,
                                                workspace=work, info=info, sketch="rows"),
            "rqr_rows_plus_pass": lambda: tsqr.rxr_cholqr(A, s, seed, Q=Q, R=R, workspace=work,
                                                          info=info, sketch="rows"),
            "rqr_gaussian_plus_pass": lambda: tsqr.rxr_cholqr(A, s, seed, Q=Q, R=R,
                                                              workspace=work, info=info),
            "cholqr2": lambda: tsqr.cholqr(A, tsqr.CHOLQR2, Q=Q, R=R, workspace=cwork,
                                           info=info),
            "scholqr3": lambda: tsqr.cholqr(A, tsqr.SCHOLQR3, -1.0, Q=Q, R=R, workspace=cwork,
                                            info=info),
        }
        row = {"kappa": kappa}
        for name, fn in methods.items():
            ms = timed(fn, args.baseline_steps, 2)
            code = int(info.item())
            o, r = gpu_metrics(A, Q, R) if code == 0 else (None, None)
            row[name] = {"ms": round(ms, 4), "info": code, "ortho": o, "residual": r}
        # Section 5.2's least-squares solver on b = A x_true (forward error against x_true)
        xt = torch.from_numpy(np.random.default_rng(3).standard_normal(n)).cuda()
        bv = (A @ xt.unsqueeze(1)).squeeze(1).contiguous()
        lwork = torch.empty(tsqr.load().tsqr_lstsq_workspace_bytes(m, n, s), dtype=torch.uint8,
                            device="cuda")
        xv = torch.empty(n, dtype=torch.float64, device="cuda")
        for sk in ("rows", "gaussian"):
            def ls(sk=sk):
                tsqr.lstsq(A, bv, s, seed, sketch=sk, x=xv, workspace=lwork, info=info)
            ms = timed(ls, args.baseline_steps, 2)
            fe = float((torch.linalg.vector_norm(xv - xt) / torch.linalg.vector_norm(xt)).item())
            row[f"lstsq_{sk}"] = {"ms": round(ms, 4), "info": int(info.item()),
                                  "forward_error": fe}
        del lwork
        base = row["rqr_rows"]["ms"]
        row["time_vs_rqr_rows"] = {k: round(row[k]["ms"] / base, 3)
                                   for k in methods if row[k]["info"] == 0}
        print(f"# baselines kappa={kappa:g}: " + ", ".join(
            f"{k} {row[k]['ms']:.3f} ms (info {row[k]['info']})" for k in methods),
            file=sys.stderr, flush=True)
        out.append(row)
        del A
        torch.cuda.empty_cache()
    return {"workload": f"tall128 shape (m={m}, n={n}, s={s})", "results": out,
            "paper": "Section 4.3, 32 processes, n=100, m=1e5: CholeskyQR2 +24% and "
                     "sCholeskyQR3 +82% time over rQR-CholeskyQR (row extraction); "
                     "CholeskyQR2 collapses beyond kappa 1e8",
            "note": "with m=2^20 the sCholeskyQR3 shift 11(mn+n(n+1))u||A||^2 bounds the "
                    "first pass's cond(Q1) by about sqrt(shift/||A||^2) kappa, which stays "
                    "below u^-1/2 (what its CholeskyQR2 needs) only up to kappa ~ 1e11; "
                    "beyond that it may break down"}


def batched_comparison(args):
    """The batched workload: 512 independent problems (m ~ U[4096, 65536], n in
    {16, 32, 64, 128}, kappa = 10^U(2,10), s = 2n, rQR + one pass, FP64).  The batch is
    planned once, autotuned, captured into one HIP graph and replayed; the baseline is the
    same factorizations issued one problem at a time through the explicit-workspace call."""
    import torch

    import paper_2111_11148_amd as tsqr
    from inputs import batched_problems, gen_matrix

    descs = batched_problems(args.batch_count, 211105)
    t0 = time.perf_counter()
    As = [tsqr.to_device_colmajor(gen_matrix(d["m"], d["n"], d["kappa"], d["gen_seed"]))
          for d in descs]
    print(f"# generated the batch ({len(descs)} problems) in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    ss = [d["s"] for d in descs]
    seeds = [d["sketch_seed"] for d in descs]
    F = sum(flops(d["m"], d["n"], d["s"], "rqr", True)["total"] for d in descs)

    b = tsqr.Batch(As, ss, seeds)
    tuning, tuned_ms = b.autotune()
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        b.run(stream=st)
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        b.run(stream=st)
    ms = timed(g.replay, args.batch_steps, 2)
    info_ok = bool(torch.all(b.info == 0).item())
    worst = 0.0
    for i in range(len(descs)):
        worst = max(worst, gpu_metrics(As[i], b.Q[i], b.R[i])[0])

    # baseline: one explicit-workspace call per problem, workspaces and outputs preallocated
    Qs = [tsqr.colmajor(A.shape[0], A.shape[1]) for A in As]
    Rs = [tsqr.colmajor(A.shape[1], A.shape[1]) for A in As]
    works = {}
    for A, s_ in zip(As, ss):
        key = (A.shape[0], A.shape[1], s_)
        if key not in works:
            works[key] = tsqr.alloc_workspace(*key)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")

    def loop():
        for i, A in enumerate(As):
            tsqr.rxr_cholqr(A, ss[i], seeds[i], Q=Qs[i], R=Rs[i],
                            workspace=works[(A.shape[0], A.shape[1], ss[i])], info=info)

    ms_loop = timed(loop, 2, 1)
    print(f"# batched: {ms:.3f} ms per batch ({len(descs) / ms * 1e3:.0f} problems/s), loop "
          f"{ms_loop:.3f} ms", file=sys.stderr, flush=True)
    del works

    # the FP32 variant: the sketch from FP32-rounded inputs, every later step FP64
    del g
    b32 = tsqr.Batch(As, ss, seeds, precision=tsqr.FP32)
    tuning32, tuned32 = b32.autotune()
    g32 = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        b32.run(stream=st)
    torch.cuda.synchronize()
    with torch.cuda.graph(g32, stream=st):
        b32.run(stream=st)
    ms32 = timed(g32.replay, args.batch_steps, 2)
    info32 = bool(torch.all(b32.info == 0).item())
    worst32 = max(gpu_metrics(As[i], b32.Q[i], b32.R[i])[0] for i in range(len(descs)))
    print(f"# batched fp32 sketch: {ms32:.3f} ms per batch ({len(descs) / ms32 * 1e3:.0f} "
          f"problems/s)", file=sys.stderr, flush=True)
    return {"workload": f"{len(descs)} uneven problems, m in [4096, 65536], n in {{16,32,64,128}}, "
                        "kappa 1e2..1e10, s = 2n, rqr + 1 pass, fp64",
            "problems_per_s": round(len(descs) / ms * 1e3, 1), "ms_per_batch": round(ms, 4),
            "gflops": round(F / ms / 1e6, 2), "flops_per_batch": F,
            "loop_problems_per_s": round(len(descs) / ms_loop * 1e3, 1),
            "loop_ms_per_batch": round(ms_loop, 4), "speedup_vs_loop": round(ms_loop / ms, 3),
            "launches_per_run": b.launches, "tuning": tuning.as_dict(),
            "autotune_ms": round(tuned_ms, 4), "graph": True, "all_info_zero": info_ok,
            "worst_ortho": worst,
            "fp32": {"problems_per_s": round(len(descs) / ms32 * 1e3, 1),
                     "ms_per_batch": round(ms32, 4), "tuning": tuning32.as_dict(),
                     "all_info_zero": info32, "worst_ortho": worst32,
                     "speedup_vs_fp64_batch": round(ms / ms32, 3)}}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", choices=["rqr", "rlu"], default="rqr")
    ap.add_argument("--cpu-sample-rows", type=int, default=1 << 20,
                    help="rows of the workload the CPU oracle is timed on (default: all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cache-dir", default=None,
                    help="directory to keep the generated input matrix between runs")
    ap.add_argument("--mixed-kappas", default="1e4,1e8,1e12",
                    help="condition numbers of the mixed-precision comparison (mixed256 "
                         "workload, m=2^20, n=256, s=512); empty to skip it")
    ap.add_argument("--mixed-steps", type=int, default=5)
    ap.add_argument("--baseline-kappas", default="1e5,1e10,1e12",
                    help="condition numbers of the comparison with CholeskyQR2 / sCholeskyQR3 "
                         "and the row-extraction sketch (m=2^20, n=128); empty to skip it")
    ap.add_argument("--baseline-steps", type=int, default=5)
    ap.add_argument("--paper-shape", type=int, default=1,
                    help="time the paper's Table scalability1 problem (m=1e7, n=100) too "
                         "(0 to skip)")
    ap.add_argument("--graph", type=int, default=1,
                    help="also time the step captured into one HIP graph (0 to skip)")
    ap.add_argument("--batch-count", type=int, default=512,
                    help="problems of the batched workload (0 to skip it)")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES bytes (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py: measures one GPU; runs over several GPUs are not supported "
              "(use --gpus 1)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2111_11148_amd as tsqr
    from inputs import WORKLOADS, gen_matrix

    if args.copy_calibration:
        nel = args.copy_calibration // 8
        x = torch.ones(nel, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nel * 8}))
        return 0

    wl = WORKLOADS["tall128"]
    m, n, s, kappa = wl.m, wl.n, wl.s, wl.kappas[0]
    seed = wl.sketch_seed
    variant = tsqr.RQR if args.variant == "rqr" else tsqr.RLU
    extra_pass = wl.extra_pass

    A_h = cached_matrix(args.cache_dir, wl.name, m, n, kappa, wl.gen_seeds[0])
    A = tsqr.to_device_colmajor(np.asarray(A_h))
    Q = tsqr.colmajor(m, n)
    R = tsqr.colmajor(n, n)
    work = tsqr.alloc_workspace(m, n, s)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")

    def step():
        tsqr.rxr_cholqr(A, s, seed, variant=variant, extra_pass=extra_pass, Q=Q, R=R,
                        workspace=work, info=info)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # per-phase breakdown: HIP events around every launch, in steps of their own
    tsqr.profile_start()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    recs_all = tsqr.profile_stop()
    phase_tot, phase_cnt = {}, {}
    for name, ms in recs_all:
        phase_tot[name] = phase_tot.get(name, 0.0) + ms
        phase_cnt[name] = phase_cnt.get(name, 0) + 1
    per_step = {k: phase_tot[k] / args.steps for k in phase_tot}
    dom = max(per_step, key=per_step.get)  # dominant kernel: largest share of the step

    # timed region: events recorded only around the dominant kernel's launches
    tsqr.profile_start(only=dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    recs = tsqr.profile_stop()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    print(f"# timed {args.steps} steps: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)

    binfo = int(info.item())
    ortho, res = gpu_metrics(A, Q, R)

    # the same step captured into one HIP graph on a side stream and replayed (no phase
    # events); every replay must reproduce the eager Q and R bit for bit
    graph = None
    if args.graph:
        Qe, Re = Q.clone(), R.clone()
        st = torch.cuda.Stream()

        def step_on(stream):
            tsqr.rxr_cholqr(A, s, seed, variant=variant, extra_pass=extra_pass, Q=Q, R=R,
                            workspace=work, info=info, stream=stream)

        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            step_on(st)
        torch.cuda.current_stream().wait_stream(st)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            step_on(st)
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        g_ms = (time.perf_counter() - t0) * 1e3 / args.steps
        same = bool(torch.equal(Q, Qe) and torch.equal(R, Re)) and int(info.item()) == 0
        graph = {"ms_per_step": round(g_ms, 4), "same_q_r_as_eager": same}
        print(f"# graph replay: {g_ms:.3f} ms/step (bitwise equal to eager: {same})",
              file=sys.stderr, flush=True)
        del Qe, Re, g

    # the dominant kernel's average launch duration, from the events of the timed steps
    dom_ms = [ms for name, ms in recs if name == dom]
    phases = {dom: sum(dom_ms) / len(dom_ms)} if dom_ms else {}

    F = flops(m, n, s, args.variant, extra_pass)
    value = F["total"] / (ms_per_step * 1e-3) / 1e9

    dom_flops = {"sketch": F["sketch"], "trsm_r0": F["trsm"], "trsm_r1": F["trsm"],
                 "trsm_r2": F["trsm"], "gram1": F["gram"], "gram2": F["gram"]}.get(dom)
    roof = None
    if dom_flops is not None and dom in phases:
        achieved = dom_flops / (phases[dom] * 1e-3) / 1e12
        traffic = load_traffic(dom, wl.name) if dom in KERNEL_SOURCES else None
        roof = {"bound": "mfma", "kernel": dom, "achieved": round(achieved, 3),
                "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": traffic,
                "avg_ms": round(phases[dom], 4)}

    # step roofline: phases separated by global dependences add up; each phase is bound
    # by max(flops / FP64 peak, algorithmic bytes / HBM bandwidth), with the algorithmic
    # bytes of the method = one read of A per phase plus the final write of Q.
    T = 8.0 * m * n
    P, BW = PEAK_FP64_TFLOPS * 1e12, PEAK_HBM_GBS * 1e9
    phase_fb = [(F["sketch"], T), (F["trsm"] + F["gram"], T)]
    if extra_pass:
        phase_fb += [(F["trsm"] + F["gram"], T), (F["trsm"], 2 * T)]
    else:
        phase_fb += [(F["trsm"], 2 * T)]
    t_roof = sum(max(fl / P, by / BW) for fl, by in phase_fb)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        ms_ = min(args.cpu_sample_rows, m)
        As = np.asfortranarray(np.asarray(A_h)[:ms_])
        # repeat the whole factorization until about 10 s of CPU work, report the mean
        reps, t_all = 0, 0.0
        while reps < 1 or (t_all < 10.0 and reps < 8):
            t0 = time.perf_counter()
            r = oracle.rxr_cholqr(As, s, seed, variant=variant, extra_pass=extra_pass)
            t_all += time.perf_counter() - t0
            reps += 1
        dt = t_all / reps
        Fs = flops(ms_, n, s, args.variant, extra_pass)["total"]
        cpu = {"value": round(Fs / dt / 1e9, 3), "unit": "GFLOP/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"first {ms_} rows of the same matrix (n={n}, s={s}), {reps} full "
                         f"factorizations, {dt:.2f} s each ({t_all:.1f} s), info={r['info']}"}

    mixed = None
    kappas = [float(k) for k in args.mixed_kappas.split(",") if k.strip()]
    if kappas:
        del A, Q, R, work
        torch.cuda.empty_cache()
        mixed = mixed_comparison(args, kappas)

    baselines = None
    bkappas = [float(k) for k in args.baseline_kappas.split(",") if k.strip()]
    if bkappas:
        torch.cuda.empty_cache()
        baselines = baselines_comparison(args, bkappas)

    paper_shaped = None
    if args.paper_shape:
        torch.cuda.empty_cache()
        paper_shaped = paper_shaped_comparison(args)

    batched = None
    if args.batch_count > 0:
        torch.cuda.empty_cache()
        batched = batched_comparison(args)

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}-{args.variant}-fp64", "m": m, "n": n, "s": s,
                   "kappa": kappa, "variant": args.variant, "extra_pass": extra_pass,
                   "flops_per_step": F["total"]},
        "roofline": roof,
        "step_roofline_frac": round(t_roof * 1e3 / ms_per_step, 4),
        "cpu_baseline": cpu,
        "ortho": ortho,
        "residual": res,
        "info": binfo,
        "phases_ms": {k: round(v, 4) for k, v in per_step.items()},
        "graph": None if graph is None else dict(
            graph, gflops=round(F["total"] / (graph["ms_per_step"] * 1e-3) / 1e9, 3)),
        "mixed_vs_fp64": mixed,
        "baselines": baselines,
        "paper_shaped": paper_shaped,
        "batched": batched,
    }
    print(json.dumps(line), flush=True)
    return 0 if binfo == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
