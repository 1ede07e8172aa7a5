"""GPU parity of the batched factorization (many uneven problems in one pass).

Each problem of a batch must meet the same bars as a single factorization: the FP64
targets (orthogonality <= 1e-12, residual <= 1e-13), R upper with a positive diagonal and
within the perturbation bound of the oracle's R; the batch must agree with the
single-problem path to that bound, replay identically from a captured HIP graph, and keep a
breakdown confined to its own problem.
"""

import numpy as np
import pytest
import torch

import oracle
import paper_2111_11148_amd as tsqr
from inputs import batched_problems, gen_matrix
from gpu_helpers import gpu_orthogonality, gpu_residual, host, rel_fro

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    tsqr.load()
    torch.cuda.synchronize()
    yield


def dev(A):
    return tsqr.to_device_colmajor(A)


# (m, n, s, kappa): every width class, ragged n, s != 2n, tiny m
SMALL = [(4096, 32, 64, 1e10), (1000, 5, 10, 1e3), (1027, 17, 34, 1e8), (6000, 128, 256, 1e12),
         (300, 1, 2, 1.0), (2500, 100, 200, 1e6), (700, 64, 96, 1e4), (129, 16, 32, 1e2),
         (5000, 33, 66, 1e9), (2048, 128, 250, 1e5), (64, 64, 128, 1e3), (3333, 48, 96, 1e7)]


def small_batch():
    mats = [gen_matrix(m, n, k, 2111050 + i) for i, (m, n, s, k) in enumerate(SMALL)]
    seeds = [11105000 + i for i in range(len(SMALL))]
    return mats, [s for (_, _, s, _) in SMALL], seeds


def test_batched_matches_oracle():
    mats, ss, seeds = small_batch()
    As = [dev(A) for A in mats]
    b = tsqr.Batch(As, ss, seeds)
    b.run()
    torch.cuda.synchronize()
    info = b.info.cpu().numpy()
    assert np.all(info == 0), info
    for i, (A, s, seed) in enumerate(zip(mats, ss, seeds)):
        Q, R = host(b.Q[i]), host(b.R[i])
        n = A.shape[1]
        kappa = SMALL[i][3]
        ortho, res = oracle.orthogonality(Q), oracle.residual(A, Q, R)
        ref = oracle.rxr_cholqr(A, s, seed)
        rd = rel_fro(R, ref["R"])
        print(f"problem {i} {A.shape} s={s} kappa={kappa:g}: ortho={ortho:.2e} res={res:.2e} "
              f"relR={rd:.2e}")
        assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
        assert ortho <= 1e-12 and res <= 1e-13
        assert rd <= 100 * n * EPS * kappa + 1e-14


def test_batched_agrees_with_single_path_and_rlu():
    mats, ss, seeds = small_batch()
    As = [dev(A) for A in mats]
    for variant in (tsqr.RQR, tsqr.RLU):
        b = tsqr.Batch(As, ss, seeds, variant=variant)
        b.run()
        for i, A in enumerate(As):
            Q1, R1, info = tsqr.rxr_cholqr(A, ss[i], seeds[i], variant=variant)
            assert int(info.item()) == 0 and int(b.info[i].item()) == 0
            n = A.shape[1]
            kappa = SMALL[i][3]
            assert rel_fro(host(b.R[i]), host(R1)) <= 200 * n * EPS * kappa + 1e-14
            if kappa <= 1e4:
                assert torch.max(torch.abs(b.Q[i] - Q1)).item() <= 200 * n * EPS * kappa


def test_batched_graph_replay_matches_eager():
    """Capture run() into a graph, replay it three times with eager work in between; every
    replay reproduces the eager result bitwise (the kernels are deterministic)."""
    mats, ss, seeds = small_batch()
    As = [dev(A) for A in mats]
    b = tsqr.Batch(As, ss, seeds)
    b.run()
    torch.cuda.synchronize()
    Q0 = [q.clone() for q in b.Q]
    R0 = [r.clone() for r in b.R]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        b.run(stream=s)  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        b.run(stream=s)
    for rep in range(3):
        for q in b.Q:
            q.zero_()
        junk = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        del junk
        for i in range(len(As)):
            assert torch.equal(b.Q[i], Q0[i]), (rep, i)
            assert torch.equal(b.R[i], R0[i]), (rep, i)
        assert torch.all(b.info == 0)


@pytest.mark.parametrize("prec", [tsqr.FP32, tsqr.BF16])
def test_batched_lowp_sketch_meets_fp64_targets(prec):
    """precision FP32/BF16: the sketch on the matrix cores (normals in the input type, A
    as its FP32 rounding: three BF16 terms on the BF16 path), every later step FP64.  Every
    problem still meets the FP64 targets and the unique R (oracle's, kappa bound): kappa
    times the FP32 unit roundoff leaves A R0^-1 within CholeskyQR2's reach for the whole
    small batch (kappa up to 1e12) with either input type."""
    mats, ss, seeds = small_batch()
    keep = list(range(len(SMALL)))
    As = [dev(mats[i]) for i in keep]
    b = tsqr.Batch(As, [ss[i] for i in keep], [seeds[i] for i in keep], precision=prec)
    b.run()
    torch.cuda.synchronize()
    assert torch.all(b.info == 0)
    for j, i in enumerate(keep):
        A = mats[i]
        n, kappa = A.shape[1], SMALL[i][3]
        Q, R = host(b.Q[j]), host(b.R[j])
        ortho, res = oracle.orthogonality(Q), oracle.residual(A, Q, R)
        ref = oracle.rxr_cholqr(A, ss[i], seeds[i])
        rd = rel_fro(R, ref["R"])
        print(f"prec={prec} problem {i} kappa={kappa:g}: ortho={ortho:.2e} res={res:.2e} "
              f"relR={rd:.2e}")
        assert ortho <= 1e-12 and res <= 1e-13
        assert rd <= 100 * n * EPS * kappa + 1e-14


def test_batched_breakdown_is_confined():
    mats, ss, seeds = small_batch()
    bad = 3
    mats[bad] = mats[bad].copy(order="F")
    mats[bad][:, 7] = 0.0
    As = [dev(A) for A in mats]
    b = tsqr.Batch(As, ss, seeds)
    b.run()
    info = b.info.cpu().numpy()
    assert info[bad] == 1008
    assert np.all(np.delete(info, bad) == 0)
    assert torch.isnan(b.Q[bad]).all() and torch.isnan(b.R[bad]).all()
    for i in range(len(As)):
        if i != bad:
            assert torch.isfinite(b.Q[i]).all()


def test_batched_without_r():
    mats, ss, seeds = small_batch()
    As = [dev(A) for A in mats]
    b1 = tsqr.Batch(As, ss, seeds)
    b1.run()
    b2 = tsqr.Batch(As, ss, seeds, want_r=False)
    b2.run()
    for i in range(len(As)):
        assert b2.R[i] is None and torch.equal(b1.Q[i], b2.Q[i])


# ------------------------------------------------------ full size: 512 uneven problems --
def test_batched_full_size_properties_and_samples():
    """The benchmark's batch (512 problems, m in [4096, 65536], n in {16,32,64,128},
    kappa in [1e2, 1e10]): every problem meets the FP64 targets on the device metrics, and
    sampled problems (one per width) match the oracle's R within the perturbation bound."""
    descs = batched_problems(512, 211105)
    As, mats_kept = [], {}
    samples = {}
    for i, d in enumerate(descs):
        if d["n"] not in samples:
            samples[d["n"]] = i
    for i, d in enumerate(descs):
        A = gen_matrix(d["m"], d["n"], d["kappa"], d["gen_seed"])
        if i in samples.values():
            mats_kept[i] = A
        As.append(dev(A))
    b = tsqr.Batch(As, [d["s"] for d in descs], [d["sketch_seed"] for d in descs])
    print(f"launches per run: {b.launches}")
    b.run()
    torch.cuda.synchronize()
    assert torch.all(b.info == 0)
    worst_o = worst_r = 0.0
    for i in range(len(descs)):
        o, r = gpu_orthogonality(b.Q[i]), gpu_residual(As[i], b.Q[i], b.R[i])
        worst_o, worst_r = max(worst_o, o), max(worst_r, r)
    print(f"worst ortho {worst_o:.2e}, worst residual {worst_r:.2e}")
    assert worst_o <= 1e-12 and worst_r <= 1e-13
    # the FP32 variant of the same batch (kappa <= 1e10: kappa u_32 <= 600)
    b32 = tsqr.Batch(As, [d["s"] for d in descs], [d["sketch_seed"] for d in descs],
                     precision=tsqr.FP32)
    b32.run()
    torch.cuda.synchronize()
    assert torch.all(b32.info == 0)
    w32 = max(gpu_orthogonality(b32.Q[i]) for i in range(len(descs)))
    r32 = max(gpu_residual(As[i], b32.Q[i], b32.R[i]) for i in range(len(descs)))
    print(f"fp32 variant: worst ortho {w32:.2e}, worst residual {r32:.2e}")
    assert w32 <= 1e-12 and r32 <= 1e-13
    del b32
    for n, i in sorted(samples.items()):
        d = descs[i]
        ref = oracle.rxr_cholqr(mats_kept[i], d["s"], d["sketch_seed"])
        rd = rel_fro(host(b.R[i]), ref["R"])
        print(f"sample {i}: m={d['m']} n={n} kappa={d['kappa']:.2g} relR={rd:.2e}")
        assert rd <= 100 * n * EPS * d["kappa"] + 1e-14
