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
    "trsm": ["paper_2111_11148_amd/csrc/k_tall.hip", "paper_2111_11148_amd/csrc/tsqr_device.hpp"],
    "gram": ["paper_2111_11148_amd/csrc/k_tall.hip", "paper_2111_11148_amd/csrc/tsqr_device.hpp"],
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
    """Orthogonality ||Q^T Q - I||_F and residual ||A - QR||_F / ||A||_F, evaluated on the
    device with double-double accumulation (the library's metric kernels)."""
    import paper_2111_11148_amd as tsqr

    return tsqr.metrics(Q, A, R)


def rel_r_diff(R_dev, R_ref) -> float:
    """||R - R_ref||_F / ||R_ref||_F against a host reference."""
    import numpy as np

    Rh = np.asarray(R_dev.cpu().numpy(), dtype=np.float64)
    return float(np.linalg.norm(Rh - R_ref) / np.linalg.norm(R_ref))


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
        row = {"kappa": kappa}
        R_or = None
        if args.mixed_oracle:
            # the FP64 oracle's R of the same matrix: every result's R is stated against it
            import oracle

            t0 = time.perf_counter()
            ref = oracle.rxr_cholqr(np.asfortranarray(A_h), s, seed, variant=oracle.RQR,
                                    extra_pass=True)
            R_or = ref["R"]
            row["fp64_oracle"] = {"seconds": round(time.perf_counter() - t0, 2),
                                  "info": int(ref["info"]), "cores": oracle.num_threads()}
            del ref
        del A_h

        def fp64():
            tsqr.rxr_cholqr(A, s, seed, Q=Q, R=R, workspace=work64, info=info)

        ms = timed(fp64, args.mixed_steps, 2)
        ortho, res = gpu_metrics(A, Q, R)
        row["fp64"] = {"ms": round(ms, 4), "gflops": round(F / ms / 1e6, 2), "ortho": ortho,
                       "residual": res, "info": int(info.item()),
                       "rel_R_vs_fp64_oracle": None if R_or is None else rel_r_diff(R, R_or),
                       "phases_ms": phases_of(fp64)}
        for name, lowp in (("fp32", tsqr.FP32), ("bf16", tsqr.BF16)):
            ws = torch.empty(tsqr.mixed_workspace_bytes(m, n, s, lowp), dtype=torch.uint8,
                             device="cuda")
            report = torch.zeros(2, dtype=torch.int32, device="cuda")

            def mixed():
                tsqr.rxr_cholqr_mixed(A, s, seed, lowp, Q=Q, R=R, workspace=ws, info=info,
                                      report=report)

            ms_m = timed(mixed, args.mixed_steps, 2)
            o_m, r_m = gpu_metrics(A, Q, R)
            ok = o_m <= 1e-12 and row["fp64"]["ortho"] <= 1e-12 and int(info.item()) == 0
            ph = phases_of(mixed)
            row[name] = {"ms": round(ms_m, 4), "gflops_equiv": round(F / ms_m / 1e6, 2),
                         "fp64_passes": int(report[0].item()),
                         "lowp_stage": bool(report[1].item()),
                         "ortho": o_m, "residual": r_m, "info": int(info.item()),
                         "rel_R_vs_fp64_oracle": None if R_or is None else rel_r_diff(R, R_or),
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

    # the batch as one persistent launch (plus the kernel that clears its counters), with
    # its own autotuned blocking, eager and captured into a graph
    bp = tsqr.Batch(As, ss, seeds)
    tuning_p, _ = bp.autotune(persistent=True)
    ms_p = timed(lambda: bp.run(persistent=True), args.batch_steps, 2)
    info_p = bool(torch.all(bp.info == 0).item())
    worst_p = max(gpu_metrics(As[i], bp.Q[i], bp.R[i])[0] for i in range(len(descs)))
    gp = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        bp.run(stream=st, persistent=True)
    torch.cuda.synchronize()
    with torch.cuda.graph(gp, stream=st):
        bp.run(stream=st, persistent=True)
    ms_pg = timed(gp.replay, args.batch_steps, 2)
    del gp
    print(f"# batched persistent: {ms_p:.3f} ms eager, {ms_pg:.3f} ms in a graph "
          f"({len(descs) / ms_pg * 1e3:.0f} problems/s), {bp.tasks} tasks",
          file=sys.stderr, flush=True)

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

    # the low-precision variants: the sketch on FP32 or BF16 matrix cores (A as its FP32
    # rounding), every later step FP64
    del g
    lowp_res = {}
    for name, prec in (("fp32", tsqr.FP32), ("bf16", tsqr.BF16)):
        bl = tsqr.Batch(As, ss, seeds, precision=prec)
        tuning_l, _ = bl.autotune()
        gl = torch.cuda.CUDAGraph()
        with torch.cuda.stream(st):
            bl.run(stream=st)
        torch.cuda.synchronize()
        with torch.cuda.graph(gl, stream=st):
            bl.run(stream=st)
        ms_l = timed(gl.replay, args.batch_steps, 2)
        info_l = bool(torch.all(bl.info == 0).item())
        worst_l = max(gpu_metrics(As[i], bl.Q[i], bl.R[i])[0] for i in range(len(descs)))
        print(f"# batched {name} sketch: {ms_l:.3f} ms per batch "
              f"({len(descs) / ms_l * 1e3:.0f} problems/s)", file=sys.stderr, flush=True)
        lowp_res[name] = {"problems_per_s": round(len(descs) / ms_l * 1e3, 1),
                          "ms_per_batch": round(ms_l, 4), "tuning": tuning_l.as_dict(),
                          "all_info_zero": info_l, "worst_ortho": worst_l,
                          "speedup_vs_fp64_batch": round(ms / ms_l, 3)}
        del gl, bl
    return {"workload": f"{len(descs)} uneven problems, m in [4096, 65536], n in {{16,32,64,128}}, "
                        "kappa 1e2..1e10, s = 2n, rqr + 1 pass, fp64",
            "problems_per_s": round(len(descs) / ms * 1e3, 1), "ms_per_batch": round(ms, 4),
            "gflops": round(F / ms / 1e6, 2), "flops_per_batch": F,
            "loop_problems_per_s": round(len(descs) / ms_loop * 1e3, 1),
            "loop_ms_per_batch": round(ms_loop, 4), "speedup_vs_loop": round(ms_loop / ms, 3),
            "launches_per_run": b.launches, "tuning": tuning.as_dict(),
            "persistent": {"ms_per_batch": round(ms_p, 4),
                           "ms_per_batch_graph": round(ms_pg, 4),
                           "problems_per_s": round(len(descs) / ms_pg * 1e3, 1),
                           "launches_per_run": 2, "tasks": bp.tasks,
                           "tuning": tuning_p.as_dict(),
                           "speedup_vs_phase_graph": round(ms / ms_pg, 3),
                           "all_info_zero": info_p, "worst_ortho": worst_p},
            "autotune_ms": round(tuned_ms, 4), "graph": True, "all_info_zero": info_ok,
            "worst_ortho": worst, "fp32": lowp_res["fp32"], "bf16": lowp_res["bf16"]}


# Kernels of the FP64 chain: the phases (library event names) each one runs under, the
# algorithmic work of one launch, and the roof that bounds it (per-unit figures:
# sketch 2smn flops over 8mn bytes, TRSM mn^2 flops over 16mn bytes, Gram
# mn(n+1) flops over 8mn bytes; at n = 128 the TRSM's 8 flop/B is below the FP64 ridge of
# 78.6 TFLOP/s / 8 TB/s = 9.8 flop/B, so it is HBM-bound, while the sketch (64 flop/B) and
# the Gram (16 flop/B) are FP64-bound).
def kernel_table(m: int, n: int, s: int, variant: str) -> dict:
    fac = "sketch_lu" if variant == "rlu" else "sketch_qr"
    return {
        "sketch": {"symbol": "k_sketch_f64", "phases": ["sketch"], "flops": 2.0 * s * m * n,
                   "bytes": 8.0 * m * n},
        "trsm": {"symbol": "k_trsm_mfma", "phases": ["trsm_r0", "trsm_r1", "trsm_r2"],
                 "flops": 1.0 * m * n * n, "bytes": 16.0 * m * n},
        "gram": {"symbol": "k_gram_f64", "phases": ["gram1", "gram2"],
                 "flops": 1.0 * m * n * (n + 1), "bytes": 8.0 * m * n},
        "sketch_factor": {"symbol": ("k_geqrf_reg / k_qr_*" if variant != "rlu"
                                     else "k_getrf_ip / k_getrf_reg / k_lu_*"),
                          "phases": [fac], "flops": None, "bytes": None},
        "potrf": {"symbol": "k_potrf_lds / k_chol_*", "phases": ["potrf1", "potrf2"],
                  "flops": n ** 3 / 3.0, "bytes": None},
        "trsm_prep": {"symbol": "k_trsm_prep",
                      "phases": ["trsm_prep_r0", "trsm_prep_r1", "trsm_prep_r2"],
                      "flops": None, "bytes": None},
    }


def roof_of(entry: dict, avg_ms: float) -> dict:
    """Roofline of one kernel from its average launch duration: bound by whichever of
    flops / FP64 peak and bytes / HBM peak is larger."""
    out = {"symbol": entry["symbol"], "avg_ms": round(avg_ms, 4)}
    fl, by = entry["flops"], entry["bytes"]
    t_f = fl / (PEAK_FP64_TFLOPS * 1e12) if fl else 0.0
    t_b = by / (PEAK_HBM_GBS * 1e9) if by else 0.0
    if fl is None or (by is None and t_f * 1e3 < 0.05 * avg_ms):
        out["bound"] = "latency"
        return out
    if t_b > t_f:
        ach = by / (avg_ms * 1e-3) / 1e9
        out.update(bound="hbm", achieved=round(ach, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                   frac=round(ach / PEAK_HBM_GBS, 4))
        if fl:
            out["mfma_frac"] = round(fl / (avg_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4)
    else:
        ach = fl / (avg_ms * 1e-3) / 1e12
        out.update(bound="mfma", achieved=round(ach, 3), peak=PEAK_FP64_TFLOPS, unit="TFLOP/s",
                   frac=round(ach / PEAK_FP64_TFLOPS, 4))
        if by:
            out["hbm_gbs"] = round(by / (avg_ms * 1e-3) / 1e9, 1)
    return out


def attainable_peaks(reps: int = 5) -> dict:
    """Measured peaks of this GPU: the best of a sweep of launch shapes of plain streaming
    kernels over 1 GiB (read, write, copy) and of independent MFMA chains (FP64, FP32,
    BF16), each timed with events on the launch stream."""
    import torch

    import paper_2111_11148_amd as tsqr

    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = {}

    def ev_time(fn):
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps  # ms

    for name, kind, moved in (("read", tsqr.PROBE_READ, nbytes),
                              ("write", tsqr.PROBE_WRITE, nbytes),
                              ("copy", tsqr.PROBE_COPY, 2 * nbytes)):
        best = (0.0, None)
        for wgs in (2, 4, 8, 16, 32):
            for unroll in ((1,) if kind == tsqr.PROBE_WRITE else (2, 4, 8)):
                for nt in ((False,) if kind == tsqr.PROBE_READ else (False, True)):
                    ms = ev_time(lambda: tsqr.probe_stream(kind, src, dst, nbytes, sink, wgs,
                                                           unroll, nt))
                    gbs = moved / (ms * 1e-3) / 1e9
                    if gbs > best[0]:
                        best = (gbs, {"wgs_per_cu": wgs, "unroll": unroll, "nontemporal": nt})
        out[f"hbm_{name}_gbs"] = round(best[0], 1)
        out[f"hbm_{name}_shape"] = best[1]
    del src, dst
    spec = {"fp64": 78.6e12, "fp64_random": 78.6e12, "fp32": 157.3e12, "bf16": 2500e12,
            "bf16_32x32": 2500e12}
    for name, kind in (("fp64", tsqr.PROBE_FP64), ("fp64_random", tsqr.PROBE_FP64_RANDOM),
                       ("fp32", tsqr.PROBE_FP32), ("bf16", tsqr.PROBE_BF16),
                       ("bf16_32x32", tsqr.PROBE_BF16_32)):
        best = (0.0, None)
        per = {3: 32768.0, 2: 16384.0}.get(kind, 2048.0)
        for w in (1, 2, 4, 8):
            for c in (4, 8, 16):
                # about 2 ms per launch at the spec rate
                per_iter = 256 * w * 4 * c * per
                iters = max(16, int(2e-3 * spec[name] / per_iter))
                fl = [0.0]

                def run():
                    fl[0] = tsqr.probe_mfma(kind, iters, sink, w, c)
                ms = ev_time(run)
                tf = fl[0] / (ms * 1e-3) / 1e12
                if tf > best[0]:
                    best = (tf, {"waves_per_simd": w, "chains": c})
        out[f"mfma_{name}_tflops"] = round(best[0], 2)
        out[f"mfma_{name}_shape"] = best[1]
    out["spec"] = {"hbm_gbs": PEAK_HBM_GBS, "mfma_fp64_tflops": PEAK_FP64_TFLOPS,
                   "mfma_fp32_tflops": 157.3, "mfma_bf16_tflops": 2500.0}
    print(f"# attainable: {out}", file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    return out


def step_t_roof(m: int, n: int, s: int, extra_pass: bool) -> float:
    """Phase-sum roofline (seconds): phases separated by global dependences add up; each
    is bound by max(flops / FP64 peak, algorithmic bytes / HBM peak), with the method's
    algorithmic bytes = one read of A per phase plus the final write of Q."""
    F = flops(m, n, s, "rqr", extra_pass)
    T = 8.0 * m * n
    P, BW = PEAK_FP64_TFLOPS * 1e12, PEAK_HBM_GBS * 1e9
    phase_fb = [(F["sketch"], T), (F["trsm"] + F["gram"], T)]
    if extra_pass:
        phase_fb += [(F["trsm"] + F["gram"], T), (F["trsm"], 2 * T)]
    else:
        phase_fb += [(F["trsm"], 2 * T)]
    return sum(max(fl / P, by / BW) for fl, by in phase_fb)


def per_kernel(recs, steps: int, table: dict) -> dict:
    """Per-step time and per-launch average of each kernel from phase records."""
    out = {}
    for key, ent in table.items():
        ms = [t for name, t in recs if name in ent["phases"]]
        if ms:
            out[key] = {"per_step_ms": sum(ms) / steps, "avg_ms": sum(ms) / len(ms),
                        "launches_per_step": len(ms) / steps}
    return out


def factor_leg(A, m, n, s, seed, variant, extra_pass, steps, label, oracle_R=None):
    """Time one whole factorization on a resident matrix; report throughput, the step
    roofline, per-kernel rooflines, device double-double metrics and, when the oracle's R
    of the same matrix is given, the relative R difference."""
    import torch

    import paper_2111_11148_amd as tsqr

    Q, R = tsqr.colmajor(m, n), tsqr.colmajor(n, n)
    work = tsqr.alloc_workspace(m, n, s)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    vcode = tsqr.RQR if variant == "rqr" else tsqr.RLU

    def step():
        tsqr.rxr_cholqr(A, s, seed, variant=vcode, extra_pass=extra_pass, Q=Q, R=R,
                        workspace=work, info=info)

    ms = timed(step, steps, 2)
    torch.cuda.synchronize()
    tsqr.profile_start()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    recs = tsqr.profile_stop()
    table = kernel_table(m, n, s, variant)
    pk = per_kernel(recs, steps, table)
    ortho, res = gpu_metrics(A, Q, R)
    F = flops(m, n, s, variant, extra_pass)["total"]
    t_roof = step_t_roof(m, n, s, extra_pass)
    out = {"workload": label, "m": m, "n": n, "s": s, "variant": variant,
           "extra_pass": extra_pass, "ms_per_step": round(ms, 4),
           "gflops": round(F / (ms * 1e-3) / 1e9, 2), "step_t_roof_ms": round(t_roof * 1e3, 4),
           "step_roofline_frac": round(t_roof * 1e3 / ms, 4), "ortho": ortho, "residual": res,
           "info": int(info.item()),
           "kernels": {k: roof_of(table[k], v["avg_ms"]) | {"per_step_ms": round(v["per_step_ms"], 4)}
                       for k, v in pk.items()}}
    if oracle_R is not None:
        out["rel_R_vs_oracle"] = rel_r_diff(R, oracle_R)
    print(f"# {label}: {ms:.3f} ms/step, ortho {ortho:.3e}, residual {res:.3e}",
          file=sys.stderr, flush=True)
    del Q, R, work
    return out


def oracle_timed(A_h, s, seed, variant, extra_pass):
    import numpy as np

    import oracle

    t0 = time.perf_counter()
    r = oracle.rxr_cholqr(np.asfortranarray(A_h), s, seed,
                          variant=oracle.RQR if variant == "rqr" else oracle.RLU,
                          extra_pass=extra_pass)
    return r, time.perf_counter() - t0


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
    ap.add_argument("--peaks", type=int, default=1,
                    help="measure attainable HBM and MFMA peaks with the probe kernels")
    ap.add_argument("--other-variant", type=int, default=1,
                    help="also time the other sketch factorization (rLU when rQR is the "
                         "headline) on the same matrix, with its oracle R difference")
    ap.add_argument("--wide", type=int, default=1,
                    help="time the wide1024 workload (m=2^18, n=1024, s=2048, plain)")
    ap.add_argument("--wide-oracle", type=int, default=1,
                    help="state the wide1024 R difference against the oracle (about a "
                         "minute of CPU work)")
    ap.add_argument("--mixed-kappas", default="1e4,1e8,1e12",
                    help="condition numbers of the mixed-precision comparison (mixed256 "
                         "workload, m=2^20, n=256, s=512); empty to skip it")
    ap.add_argument("--mixed-steps", type=int, default=5)
    ap.add_argument("--mixed-oracle", type=int, default=1,
                    help="state each mixed256 result's R difference against the FP64 oracle")
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
    from inputs import WORKLOADS

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

    # per-kernel breakdown: HIP events around every launch, in steps of their own
    tsqr.profile_start()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    recs_all = tsqr.profile_stop()
    phase_tot = {}
    for name, ms in recs_all:
        phase_tot[name] = phase_tot.get(name, 0.0) + ms
    per_step = {k: phase_tot[k] / args.steps for k in phase_tot}
    table = kernel_table(m, n, s, args.variant)
    pk = per_kernel(recs_all, args.steps, table)
    # dominant kernel: the largest share of the step, all of its launches together
    dom = max(pk, key=lambda k: pk[k]["per_step_ms"])

    # timed region: events recorded only around the dominant kernel's launches
    tsqr.profile_start(only=",".join(table[dom]["phases"]))
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
    dom_ms = [t for name, t in recs if name in table[dom]["phases"]]
    dom_avg = sum(dom_ms) / len(dom_ms)
    roof = roof_of(table[dom], dom_avg)
    roof["kernel"] = dom
    roof["launches_per_step"] = round(len(dom_ms) / args.steps, 2)
    roof["traffic"] = load_traffic(dom, wl.name) if dom in KERNEL_SOURCES else None
    kernels = {k: roof_of(table[k], v["avg_ms"]) | {"per_step_ms": round(v["per_step_ms"], 4)}
               for k, v in pk.items()}

    F = flops(m, n, s, args.variant, extra_pass)
    value = F["total"] / (ms_per_step * 1e-3) / 1e9
    t_roof = step_t_roof(m, n, s, extra_pass)

    peaks = attainable_peaks() if args.peaks else None
    if peaks:
        # the same achieved rate against what the probe kernels reach on this GPU
        if roof.get("bound") == "hbm":
            roof["frac_of_attainable_copy"] = round(roof["achieved"] / peaks["hbm_copy_gbs"], 4)
        elif roof.get("bound") == "mfma":
            # the method's operands are data, not constants: the random-operand rate
            roof["frac_of_attainable_mfma"] = round(
                roof["achieved"] / peaks["mfma_fp64_random_tflops"], 4)

    cpu = None
    rel_R = None
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
        if ms_ == m:
            rel_R = rel_r_diff(R, r["R"])
        del As, r

    other = None
    if args.other_variant:
        ov = "rlu" if args.variant == "rqr" else "rqr"
        R_o = None
        if not args.no_cpu_baseline:
            ro, t_o = oracle_timed(A_h, s, seed, ov, extra_pass)
            R_o = ro["R"]
        other = factor_leg(A, m, n, s, seed, ov, extra_pass, args.steps,
                           f"{wl.name}-{ov}-fp64", oracle_R=R_o)
        if R_o is not None:
            other["oracle_seconds"] = round(t_o, 2)

    del A, Q, R, work
    torch.cuda.empty_cache()

    wide = None
    if args.wide:
        ww = WORKLOADS["wide1024"]
        Aw_h = cached_matrix(args.cache_dir, ww.name, ww.m, ww.n, ww.kappas[0], ww.gen_seeds[0])
        Aw = tsqr.to_device_colmajor(np.asarray(Aw_h))
        R_w, t_w = None, None
        if args.wide_oracle and not args.no_cpu_baseline:
            rw, t_w = oracle_timed(Aw_h, ww.s, ww.sketch_seed, "rqr", ww.extra_pass)
            R_w = rw["R"]
            del rw
        wide = factor_leg(Aw, ww.m, ww.n, ww.s, ww.sketch_seed, "rqr", ww.extra_pass,
                          5, f"{ww.name}-rqr-fp64", oracle_R=R_w)
        if t_w is not None:
            wide["oracle_seconds"] = round(t_w, 2)
        del Aw, Aw_h
        torch.cuda.empty_cache()

    mixed = None
    kappas = [float(k) for k in args.mixed_kappas.split(",") if k.strip()]
    if kappas:
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
        "step_t_roof_ms": round(t_roof * 1e3, 4),
        "kernels": kernels,
        "attainable_peaks": peaks,
        "cpu_baseline": cpu,
        "ortho": ortho,
        "residual": res,
        "rel_R_vs_oracle": rel_R,
        "info": binfo,
        "phases_ms": {k: round(v, 4) for k, v in per_step.items()},
        "graph": None if graph is None else dict(
            graph, gflops=round(F["total"] / (graph["ms_per_step"] * 1e-3) / 1e9, 3)),
        "other_variant": other,
        "wide1024": wide,
        "mixed_vs_fp64": mixed,
        "baselines": baselines,
        "paper_shaped": paper_shaped,
        "batched": batched,
    }
    print(json.dumps(line), flush=True)
    return 0 if binfo == 0 else 1


if __name__ == "__main__":
    sys.exit(main())
