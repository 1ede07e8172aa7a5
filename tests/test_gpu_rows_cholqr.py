"""GPU parity of the row-extraction sketch (Section 2.3, "Row Extraction") and of the
CholeskyQR family the paper compares against (Section 2.1: CholeskyQR, CholeskyQR2,
shifted CholeskyQR3), through the C ABI, against the CPU oracle.

The row sample is a copy, so it is compared bit for bit.  The factorizations are compared
as the FP64 method is: the targets (||Q^T Q - I||_F <= 1e-12, residual <= 1e-13) where the
algorithm is meant to reach them, R within the perturbation bound c n eps kappa of the
oracle's R, and breakdowns with the oracle's stage.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2111_11148_amd as tsqr
from inputs import gen_matrix
from gpu_helpers import gpu_orthogonality, gpu_residual, host, rel_fro

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
EPS = 2.0 ** -52


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    tsqr.load()
    torch.cuda.synchronize()
    yield


def dev(A, ld=None):
    return tsqr.to_device_colmajor(A, ld=ld)


# ------------------------------------------------------------------- row extraction --
@pytest.mark.parametrize("m,n,s,seed", [(4096, 32, 64, 1), (1000, 5, 7, 2), (777, 1, 1, 3),
                                        (200000, 17, 40, 4), (3 * (1 << 21) + 5, 1, 300, 5)])
def test_sketch_rows_bit_exact(m, n, s, seed):
    rng = np.random.default_rng(seed)
    A = np.asfortranarray(rng.standard_normal((m, n)))
    Bg = host(tsqr.sketch_rows(dev(A, ld=m + 3), s, seed))
    Bo = oracle.sketch_rows(A, s, seed)
    assert np.array_equal(Bg, Bo)


@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
@pytest.mark.parametrize("m,n,s,kappa", [(4096, 32, 64, 1e4), (4096, 32, 64, 1e14),
                                         (1027, 17, 40, 1e10), (6000, 128, 256, 1e12),
                                         (300, 1, 2, 1.0)])
def test_rows_driver_parity(variant, m, n, s, kappa):
    A = gen_matrix(m, n, kappa, 2111060 + m + n)
    seed = 11106 + n
    Qd, Rd, info = tsqr.rxr_cholqr(dev(A), s, seed, variant=variant, sketch="rows")
    assert int(info.item()) == 0
    ref = oracle.rxr_cholqr(A, s, seed, variant=variant, sketch="rows")
    assert ref["info"] == 0
    Q, R = host(Qd), host(Rd)
    ortho, res = oracle.orthogonality(Q), oracle.residual(A, Q, R)
    rd = rel_fro(R, ref["R"])
    print(f"rows variant={variant} m={m} n={n} kappa={kappa:g}: ortho={ortho:.2e} "
          f"res={res:.2e} relR={rd:.2e}")
    assert ortho <= 1e-12 and res <= 1e-13
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    assert rd <= 100 * n * EPS * kappa + 1e-14


def test_rows_worst_case_identity_block():
    """[I_n; 0] with s << m: the sample misses some of the first n rows, the small
    factorization breaks down (stage 1, as in the oracle) and Q, R are NaN."""
    m, n, s = 4096, 8, 16
    A = np.zeros((m, n), order="F")
    A[:n, :n] = np.eye(n)
    ref = oracle.rxr_cholqr(A, s, 3, sketch="rows")
    Qd, Rd, info = tsqr.rxr_cholqr(dev(A), s, 3, sketch="rows")
    assert ref["info"] // 1000 == 1 and int(info.item()) // 1000 == 1
    assert torch.isnan(Qd).all() and torch.isnan(Rd).all()


def test_rows_deterministic_and_rless():
    A = dev(gen_matrix(20000, 64, 1e10, 8))
    Q1, R1, _ = tsqr.rxr_cholqr(A, 128, 9, sketch="rows")
    Q2, R2, _ = tsqr.rxr_cholqr(A, 128, 9, sketch="rows")
    Q3, R3, _ = tsqr.rxr_cholqr(A, 128, 9, sketch="rows", want_r=False)
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2) and R3 is None and torch.equal(Q1, Q3)


def test_rows_tall128_full_size():
    """The benchmark's 2^20 x 128, kappa 1e14 matrix with the row sample: the FP64 targets
    on the device metrics, and the same unique R as the Gaussian-sketch path (both within
    the kappa u perturbation bound)."""
    m, n, s = 1 << 20, 128, 256
    A = gen_matrix(m, n, 1e14, 211102)
    Ad = dev(A)
    del A
    Qd, Rd, info = tsqr.rxr_cholqr(Ad, s, 11102, sketch="rows")
    assert int(info.item()) == 0
    o, r = gpu_orthogonality(Qd), gpu_residual(Ad, Qd, Rd)
    Qg, Rg, infog = tsqr.rxr_cholqr(Ad, s, 11102)
    assert int(infog.item()) == 0
    rd = rel_fro(host(Rd), host(Rg))
    print(f"rows tall128: ortho={o:.2e} res={r:.2e} rel R vs gaussian={rd:.2e}")
    assert o <= 1e-12 and r <= 1e-13
    assert rd <= 200 * n * EPS * 1e14


# -------------------------------------------------------------------- CholeskyQR family --
@pytest.mark.parametrize("algo,kappa,shift", [(tsqr.CHOLQR2, 1e3, -1.0), (tsqr.CHOLQR2, 1e6, -1.0),
                                              (tsqr.SCHOLQR3, 1e12, -1.0),
                                              (tsqr.SCHOLQR3, 1e12, 1e-15),
                                              (tsqr.SCHOLQR3, 1e4, -1.0)])
@pytest.mark.parametrize("m,n", [(4096, 16), (2049, 33)])
def test_cholqr_family_meets_targets(algo, kappa, shift, m, n):
    A = gen_matrix(m, n, kappa, 2111070 + m + n)
    Qd, Rd, info = tsqr.cholqr(dev(A, ld=m + 1), algo, shift)
    npass = 2 if algo == tsqr.CHOLQR2 else 3
    Qo, Ro, io = oracle.cholqr_n(A, npass, shift if algo == tsqr.SCHOLQR3 else 0.0)
    assert io == 0 and int(info.item()) == 0
    Q, R = host(Qd), host(Rd)
    ortho, res = oracle.orthogonality(Q), oracle.residual(A, Q, R)
    rd = rel_fro(R, Ro)
    print(f"algo={algo} m={m} n={n} kappa={kappa:g} shift={shift:g}: ortho={ortho:.2e} "
          f"res={res:.2e} relR={rd:.2e}")
    assert ortho <= 1e-12 and res <= 1e-13
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    assert rd <= 100 * n * EPS * kappa + 1e-14


@pytest.mark.parametrize("kappa", [1e2, 1e5])
def test_cholqr_single_pass_matches_oracle(kappa):
    """Plain CholeskyQR: Q loses orthogonality like kappa^2 u on both sides; R agrees with
    the oracle's within the perturbation bound of the Gram matrix (kappa^2 n eps)."""
    m, n = 4096, 16
    A = gen_matrix(m, n, kappa, 5)
    Qd, Rd, info = tsqr.cholqr(dev(A), tsqr.CHOLQR)
    Qo, Ro, io = oracle.cholqr_n(A, 1)
    assert io == 0 and int(info.item()) == 0
    Q, R = host(Qd), host(Rd)
    assert rel_fro(R, Ro) <= 100 * n * EPS * kappa ** 2
    assert oracle.orthogonality(Q) <= 100 * kappa ** 2 * EPS + 1e-14
    assert oracle.residual(A, Q, R) <= 1e-13


def test_cholqr2_collapses_like_the_oracle():
    """kappa 1e12 >> u^-1/2: CholeskyQR2's first Cholesky breaks down on both sides with the
    same stage; sCholeskyQR3 with the suggested shift succeeds on the same matrix."""
    m, n = 4096, 16
    A = gen_matrix(m, n, 1e12, 6)
    Qo, Ro, io = oracle.cholqr_n(A, 2)
    Qd, Rd, info = tsqr.cholqr(dev(A), tsqr.CHOLQR2)
    assert io != 0 and int(info.item()) // 1000 == io // 1000
    assert torch.isnan(Qd).all() and torch.isnan(Rd).all()
    Q3, R3, i3 = tsqr.cholqr(dev(A), tsqr.SCHOLQR3, -1.0)
    assert int(i3.item()) == 0
    assert oracle.orthogonality(host(Q3)) <= 1e-12


def test_cholqr_full_size():
    """2^20 x 128 (the benchmark shape): CholeskyQR2 at kappa 1e5 and sCholeskyQR3 (suggested
    shift) at kappa 1e8 meet the FP64 targets on the device metrics."""
    m, n = 1 << 20, 128
    for algo, kappa in ((tsqr.CHOLQR2, 1e5), (tsqr.SCHOLQR3, 1e8)):
        A = gen_matrix(m, n, kappa, 211107)
        Ad = dev(A)
        del A
        Qd, Rd, info = tsqr.cholqr(Ad, algo, -1.0)
        assert int(info.item()) == 0
        o, r = gpu_orthogonality(Qd), gpu_residual(Ad, Qd, Rd)
        print(f"algo={algo} kappa={kappa:g} full size: ortho={o:.2e} res={r:.2e}")
        assert o <= 1e-12 and r <= 1e-13
        del Ad, Qd, Rd
        torch.cuda.empty_cache()
