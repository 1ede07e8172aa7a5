"""The batch as one persistent launch (tsqr_batched_run_persistent): the same bars as the
phase-by-phase batch.  Every problem meets the FP64 targets and the oracle's R within the
perturbation bound; the persistent result agrees with the phase-by-phase one to that bound
(its reductions run in another fixed order); runs repeat bit for bit, also from a captured
graph; a breakdown stays confined to its problem."""

import numpy as np
import pytest
import torch

import oracle
import paper_2111_11148_amd as tsqr
from gpu_helpers import host, rel_fro
from inputs import batched_problems, gen_matrix

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -52

# (m, n, s, kappa): every width class, ragged n, s != 2n, s = 512, tiny m
SMALL = [(4096, 32, 64, 1e10), (1000, 5, 10, 1e3), (1027, 17, 34, 1e8), (6000, 128, 256, 1e12),
         (300, 1, 2, 1.0), (2500, 100, 200, 1e6), (700, 64, 96, 1e4), (129, 16, 32, 1e2),
         (5000, 33, 66, 1e9), (2048, 128, 250, 1e5), (64, 64, 128, 1e3), (3333, 48, 512, 1e7)]


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    tsqr.load()
    torch.cuda.synchronize()
    yield


def small_batch(cases=SMALL):
    mats = [gen_matrix(m, n, k, 2111070 + i) for i, (m, n, s, k) in enumerate(cases)]
    seeds = [11107000 + i for i in range(len(cases))]
    return mats, [s for (_, _, s, _) in cases], seeds


def test_persistent_tiny_batch_first():
    """Two problems, then three: the smallest runs of the schedule (printed before each)."""
    for cases in ([(300, 8, 16, 1e3), (1000, 32, 64, 1e6)],
                  [(4096, 128, 256, 1e8), (129, 1, 1, 1.0), (2000, 64, 128, 1e4)]):
        mats, ss, seeds = small_batch(cases)
        print(f"persistent batch of {len(cases)}: {cases}", flush=True)
        b = tsqr.Batch([tsqr.to_device_colmajor(A) for A in mats], ss, seeds)
        b.run(persistent=True)
        torch.cuda.synchronize()
        assert np.all(b.info.cpu().numpy() == 0)
        for i, A in enumerate(mats):
            Q, R = host(b.Q[i]), host(b.R[i])
            assert oracle.orthogonality(Q) <= 1e-12 and oracle.residual(A, Q, R) <= 1e-13


@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
def test_persistent_matches_oracle_and_phase_schedule(variant):
    mats, ss, seeds = small_batch()
    As = [tsqr.to_device_colmajor(A) for A in mats]
    b = tsqr.Batch(As, ss, seeds, variant=variant)
    print(f"tasks {b.tasks}, launches of the phase schedule {b.launches}", flush=True)
    b.run(persistent=True)
    torch.cuda.synchronize()
    assert np.all(b.info.cpu().numpy() == 0)
    Qp = [host(q) for q in b.Q]
    Rp = [host(r) for r in b.R]
    b.run()  # the phase-by-phase schedule of the same plan
    torch.cuda.synchronize()
    for i, (A, s, seed) in enumerate(zip(mats, ss, seeds)):
        n, kappa = A.shape[1], SMALL[i][3]
        ortho, res = oracle.orthogonality(Qp[i]), oracle.residual(A, Qp[i], Rp[i])
        ref = oracle.rxr_cholqr(A, s, seed, variant=variant)
        rd = rel_fro(Rp[i], ref["R"])
        rp = rel_fro(Rp[i], host(b.R[i]))
        print(f"problem {i} {A.shape} s={s} kappa={kappa:g}: ortho={ortho:.2e} res={res:.2e} "
              f"relR(oracle)={rd:.2e} relR(phase schedule)={rp:.2e}")
        assert np.all(np.tril(Rp[i], -1) == 0) and np.all(np.diag(Rp[i]) > 0)
        assert ortho <= 1e-12 and res <= 1e-13
        assert rd <= 100 * n * EPS * kappa + 1e-14
        assert rp <= 200 * n * EPS * kappa + 1e-14


def test_persistent_repeats_and_graph_replay():
    mats, ss, seeds = small_batch()
    As = [tsqr.to_device_colmajor(A) for A in mats]
    b = tsqr.Batch(As, ss, seeds)
    b.run(persistent=True)
    torch.cuda.synchronize()
    Q0 = [q.clone() for q in b.Q]
    R0 = [r.clone() for r in b.R]
    b.run(persistent=True)
    torch.cuda.synchronize()
    for i in range(len(As)):
        assert torch.equal(b.Q[i], Q0[i]) and torch.equal(b.R[i], R0[i]), i
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        b.run(stream=st, persistent=True)
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        b.run(stream=st, persistent=True)
    for rep in range(3):
        for q in b.Q:
            q.zero_()
        b.info.fill_(-3)
        junk = torch.randn(1000, 1000, device="cuda") @ torch.randn(1000, 1000, device="cuda")
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        del junk
        assert torch.all(b.info == 0), rep
        for i in range(len(As)):
            assert torch.equal(b.Q[i], Q0[i]) and torch.equal(b.R[i], R0[i]), (rep, i)
        b.run()  # eager phase-schedule work between the replays
        torch.cuda.synchronize()


def test_persistent_breakdown_is_confined():
    mats, ss, seeds = small_batch()
    bad = 3
    mats[bad] = mats[bad].copy(order="F")
    mats[bad][:, 7] = 0.0
    As = [tsqr.to_device_colmajor(A) for A in mats]
    b = tsqr.Batch(As, ss, seeds)
    b.run(persistent=True)
    torch.cuda.synchronize()
    info = b.info.cpu().numpy()
    assert info[bad] == 1008
    assert np.all(np.delete(info, bad) == 0)
    assert torch.isnan(b.Q[bad]).all() and torch.isnan(b.R[bad]).all()
    for i in range(len(As)):
        if i != bad:
            assert torch.isfinite(b.Q[i]).all()


@pytest.mark.parametrize("prec", [tsqr.FP32, tsqr.BF16])
def test_persistent_lowp_sketch(prec):
    """Low-precision sketch in the persistent kernel: the FP64 targets and the oracle's R
    within the kappa bound on every problem of the small batch (kappa up to 1e12), with
    either input type (A enters the sketch as its FP32 rounding)."""
    mats, ss, seeds = small_batch()
    keep = list(range(len(SMALL)))
    As = [tsqr.to_device_colmajor(mats[i]) for i in keep]
    b = tsqr.Batch(As, [ss[i] for i in keep], [seeds[i] for i in keep], precision=prec)
    b.run(persistent=True)
    torch.cuda.synchronize()
    assert torch.all(b.info == 0)
    for j, i in enumerate(keep):
        A = mats[i]
        n, kappa = A.shape[1], SMALL[i][3]
        Q, R = host(b.Q[j]), host(b.R[j])
        ortho, res = oracle.orthogonality(Q), oracle.residual(A, Q, R)
        ref = oracle.rxr_cholqr(A, ss[i], seeds[i])
        rd = rel_fro(R, ref["R"])
        print(f"prec={prec} problem {i}: ortho={ortho:.2e} res={res:.2e} relR={rd:.2e}")
        assert ortho <= 1e-12 and res <= 1e-13
        assert rd <= 100 * n * EPS * kappa + 1e-14


def test_persistent_full_size_batch():
    """The benchmark's 512 uneven problems in one persistent launch: every problem meets
    the FP64 targets (device double-double metrics), and agrees with the phase schedule."""
    descs = batched_problems(512, 211105)
    As = [tsqr.to_device_colmajor(gen_matrix(d["m"], d["n"], d["kappa"], d["gen_seed"]))
          for d in descs]
    b = tsqr.Batch(As, [d["s"] for d in descs], [d["sketch_seed"] for d in descs])
    print(f"tasks {b.tasks}", flush=True)
    b.run(persistent=True)
    torch.cuda.synchronize()
    assert torch.all(b.info == 0)
    Rp = [r.clone() for r in b.R]
    worst_o = worst_r = 0.0
    for i in range(len(descs)):
        o, r = tsqr.metrics(b.Q[i], As[i], b.R[i])
        worst_o, worst_r = max(worst_o, o), max(worst_r, r)
    print(f"worst ortho {worst_o:.2e}, worst residual {worst_r:.2e}")
    assert worst_o <= 1e-12 and worst_r <= 1e-13
    b.run()
    torch.cuda.synchronize()
    for i, d in enumerate(descs):
        rd = float(torch.linalg.matrix_norm(Rp[i] - b.R[i]) / torch.linalg.matrix_norm(b.R[i]))
        assert rd <= 200 * d["n"] * EPS * d["kappa"] + 1e-14, (i, rd)
