"""Pins of the oracle's row-extraction sketch (Section 2.3, "Row Extraction", with the
sampling of Theorem "Equal Probability Case") and of the suggested sCholeskyQR3 shift
(Section 2.1), against things other than the oracle itself: distribution tests of the
drawn rows, NumPy fancy indexing, LAPACK's R factor, the paper's worst case [I; 0], and
the shift's first-order effect on the first Cholesky factor."""
import math

import numpy as np
import pytest
import scipy.stats

import oracle
from inputs import gen_matrix
from paper_claims import paper_claims

U64 = 2.0 ** -53


def signfix(Rm):
    d = np.sign(np.diag(Rm))
    d[d == 0] = 1
    return d[:, None] * Rm


@pytest.mark.parametrize("m", [1, 7, 1000, 1 << 20, 3 * (1 << 35)])
def test_sample_rows_in_range_and_uniform(m):
    """Every index lies in [0, m); over 16 equal bins of [0, m) the counts pass a
    chi-square test (m = 3 * 2^35 would fail if only 32 random bits were used)."""
    s = 64000
    r = oracle.sample_rows(m, s, 2111)
    assert r.min() >= 0 and r.max() < m
    if m >= 1000:
        bins = np.minimum((r.astype(np.float64) * 16 / m).astype(np.int64), 15)
        counts = np.bincount(bins, minlength=16)
        p = scipy.stats.chisquare(counts).pvalue
        assert p > 1e-4, counts
        # consecutive draws are independent: no lag-1 correlation
        x = r.astype(np.float64) / m
        assert abs(np.corrcoef(x[:-1], x[1:])[0, 1]) < 0.02


def test_sample_rows_seed_and_prefix():
    """Different seeds give different draws; draw i does not depend on s (a prefix)."""
    a = oracle.sample_rows(10 ** 6, 100, 1)
    b = oracle.sample_rows(10 ** 6, 100, 2)
    c = oracle.sample_rows(10 ** 6, 40, 1)
    assert not np.array_equal(a, b)
    assert np.array_equal(a[:40], c)


def test_sketch_rows_is_a_row_gather():
    A = gen_matrix(3000, 12, 1e3, 4)
    B = oracle.sketch_rows(A, 50, 9)
    rows = oracle.sample_rows(3000, 50, 9)
    assert np.array_equal(B, A[rows, :])


@pytest.mark.parametrize("variant", [oracle.RQR, oracle.RLU])
@pytest.mark.parametrize("kappa", [1e2, 1e8, 1e13])
def test_rows_driver_is_a_qr_factorization(variant, kappa):
    """With row extraction the method still returns the unique positive-diagonal R of A
    (LAPACK's, to kappa u), an orthonormal Q and a u-level residual; and the row sample
    preconditions: cond(A R0^-1) is O(1) for an incoherent A (Section 3)."""
    m, n, s = 4096, 24, 48
    A = gen_matrix(m, n, kappa, 77)
    r = oracle.rxr_cholqr(A, s, 5, variant=variant, sketch="rows")
    assert r["info"] == 0
    assert oracle.orthogonality(r["Q"]) <= 1e-13
    assert oracle.residual(A, r["Q"], r["R"]) <= 1e-14
    Rl = signfix(np.linalg.qr(A, mode="r"))
    assert np.linalg.norm(r["R"] - Rl) / np.linalg.norm(Rl) <= 4 * n * kappa * U64 + 1e-14
    A1 = np.linalg.solve(r["R0"].T, A.T).T
    assert np.linalg.cond(A1) < 50.0


def test_rows_worst_case_identity_block():
    """The paper's extreme case A = [I_n; 0]: a row sample of size s << m misses most of
    the first n rows, so the sampled matrix is rank deficient and the method reports a
    breakdown of the small factorization (stage 1) with NaN outputs."""
    m, n, s = 4096, 8, 16
    A = np.zeros((m, n), order="F")
    A[:n, :n] = np.eye(n)
    rows = oracle.sample_rows(m, s, 3)
    assert len(set(rows.tolist()) & set(range(n))) < n
    r = oracle.rxr_cholqr(A, s, 3, sketch="rows")
    assert r["info"] // 1000 == 1
    assert np.isnan(r["Q"]).all() and np.isnan(r["R"]).all()


def test_suggested_shift_first_factor():
    """shift < 0 adds 11 (mn + n(n+1)) u ||A^T A||_F to the Gram diagonal (Section 2.1),
    with u the machine precision the paper fixes in Section 4.1 (read from the golden
    file, not from the oracle).  One shifted pass equals the pass with that shift given
    explicitly, and is told apart from the pass with u off by a factor of two either way
    (the unit roundoff 2^-53 in place of 2^-52 is exactly that mistake)."""
    u = paper_claims()["u"]
    assert u == 2.0 ** -52
    m, n = 2048, 16
    A = gen_matrix(m, n, 1e3, 8)
    G = A.T @ A
    sh = 11.0 * (m * n + n * (n + 1)) * u * np.linalg.norm(G)
    _, Ra, ia = oracle.cholqr_n(A, 1, shift=-1.0)
    _, Rb, ib = oracle.cholqr_n(A, 1, shift=sh)
    _, Rh, ih = oracle.cholqr_n(A, 1, shift=sh / 2)
    _, Rd, idd = oracle.cholqr_n(A, 1, shift=2 * sh)
    assert ia == ib == ih == idd == 0
    d_ab = np.linalg.norm(Ra - Rb) / np.linalg.norm(Rb)
    # R^T R = G + shift I: halving or doubling the shift moves R by the first-order amount
    # (shift / 2) / ||G|| times a factor of order one, far above d_ab
    d_ah = np.linalg.norm(Ra - Rh) / np.linalg.norm(Rh)
    d_ad = np.linalg.norm(Ra - Rd) / np.linalg.norm(Rd)
    first_order = 0.5 * sh / np.linalg.norm(G)
    assert d_ab < 1e-14
    assert d_ah > 0.05 * first_order and d_ad > 0.05 * first_order
    assert d_ab < 1e-3 * min(d_ah, d_ad)


def test_scholqr3_with_suggested_shift_and_cholqr2_collapse():
    """Section 4.3: CholeskyQR2 collapses past kappa 1e8 while sCholeskyQR3 (suggested
    shift) still returns an orthonormal Q with a u-level residual."""
    A = gen_matrix(4096, 16, 1e12, 6)
    Q2, _, i2 = oracle.cholqr_n(A, 2)
    assert i2 != 0 or oracle.orthogonality(Q2) > 1e-6
    Q3, R3, i3 = oracle.cholqr_n(A, 3, shift=-1.0)
    assert i3 == 0
    assert oracle.orthogonality(Q3) < 1e-13
    assert oracle.residual(A, Q3, R3) < 1e-14


# ---------------------------------------------------------------- least squares ----
@pytest.mark.parametrize("sketch", ["gaussian", "rows"])
@pytest.mark.parametrize("variant", [oracle.RQR, oracle.RLU])
@pytest.mark.parametrize("kappa", [1e3, 1e10])
def test_lstsq_against_lapack(sketch, variant, kappa):
    """Section 5.2's solver: a consistent system is solved to its forward-error level
    kappa u (with constant 100), and an inconsistent one agrees with LAPACK's
    QR-based least-squares solution to the same level."""
    m, n = 4096, 32
    A = gen_matrix(m, n, kappa, 3)
    rng = np.random.default_rng(1)
    xt = rng.standard_normal(n)
    x, info = oracle.lstsq(A, A @ xt, 64, 5, variant=variant, sketch=sketch)
    assert info == 0
    assert np.linalg.norm(x - xt) / np.linalg.norm(xt) <= 100 * kappa * U64
    b = A @ xt + 1e-3 * rng.standard_normal(m)
    x2, info = oracle.lstsq(A, b, 64, 5, variant=variant, sketch=sketch)
    xl = np.linalg.lstsq(A, b, rcond=None)[0]
    assert info == 0
    assert np.linalg.norm(x2 - xl) / np.linalg.norm(xl) <= 100 * kappa * U64


def test_lstsq_closed_form():
    """A = [D; 0] with D diagonal: x = b[:n] / diag(D) whatever the sketch and its R."""
    m, n = 512, 8
    A = np.zeros((m, n), order="F")
    d = 2.0 ** np.arange(n)
    A[:n, :n] = np.diag(d)
    b = np.arange(1.0, m + 1.0)
    x, info = oracle.lstsq(A, b, 16, 2)
    assert info == 0
    assert np.allclose(x, b[:n] / d, rtol=1e-14, atol=0)
