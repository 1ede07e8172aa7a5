"""Pins of the oracle's mixed-precision routines against things other than themselves.

The low-precision steps are pinned by: torch's own FP32 -> BF16 conversion (round to
nearest even), exact integer arithmetic (inputs that every type represents, so the rounded
and the exact results coincide), reduction to the pinned FP64 routines when rounding is
the identity, and LAPACK's triangular inverse.  The mixed driver is pinned by the
invariants of a QR factorization and by LAPACK's R factor within the perturbation bound.
"""
import math

import numpy as np
import pytest
import scipy.linalg
import torch

import oracle
from inputs import gen_matrix

FP32, BF16 = oracle.FP32, oracle.BF16
U64 = 2.0 ** -53


def F(x):
    return np.asfortranarray(x, dtype=np.float64)


def torch_round(x, prec):
    t = torch.as_tensor(np.asarray(x, dtype=np.float64)).to(torch.float32)
    if prec == BF16:
        t = t.to(torch.bfloat16).to(torch.float32)
    return t.to(torch.float64).numpy()


def signfix(Rm):
    d = np.sign(np.diag(Rm))
    d[d == 0] = 1
    return d[:, None] * Rm


# ------------------------------------------------------------------------- rounding --
def test_round_bf16_matches_torch():
    rng = np.random.default_rng(5)
    xs = list(rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000))
    # ties at the BF16 rounding point: 1 + 2^-8 (tie, even down), 1 + 3*2^-8 (tie, up)
    xs += [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 1.0 + 2.0 ** -8 + 2.0 ** -20,
           0.0, -0.0, 1e-40, -3e-39, 3.3e38, 1e39, float("inf"), float("-inf")]
    for x in xs:
        got = oracle.round_bf16(x)
        exp = float(torch_round(x, BF16))
        assert got == exp or (math.isnan(got) and math.isnan(exp)), (x, got, exp)
    assert math.isnan(oracle.round_bf16(float("nan")))


def test_round_fp32_matches_numpy():
    rng = np.random.default_rng(6)
    with np.errstate(over="ignore"):
        for x in rng.standard_normal(5000) * 10.0 ** rng.integers(-40, 40, 5000):
            assert oracle.round_fp32(x) == float(np.float32(x))


# ------------------------------------------------------------------------- triangle --
@pytest.mark.parametrize("n", [1, 7, 33])
def test_trtri_matches_lapack(n):
    rng = np.random.default_rng(n)
    T = np.triu(rng.standard_normal((n, n))) + 4 * np.eye(n)
    X = oracle.trtri_upper(F(T))
    exp = scipy.linalg.solve_triangular(T, np.eye(n), lower=False)
    assert np.array_equal(np.tril(X, -1), np.zeros((n, n)))
    assert np.abs(X - exp).max() <= 64 * n * U64 * np.abs(exp).max()
    assert np.abs(T @ X - np.eye(n)).max() <= 64 * n * U64 * np.abs(T).max() * np.abs(X).max()


# ------------------------------------------------------------------------ sketch ----
def test_sketch_lowp_reduces_to_fp64_sketch_on_representable_input():
    """With A exactly representable in BF16 and the normals already FP32 numbers, only the
    rounding of the normals separates the low-precision sketch from the FP64 one."""
    m, n, s, seed = 300, 5, 16, 11104
    rng = np.random.default_rng(0)
    A = F(rng.integers(-128, 128, size=(m, n)) * 2.0 ** -4)  # 8-bit significands
    Z = oracle.sketch_normals(seed, 0, s, 0, m)
    B64 = oracle.sketch_apply(A, s, seed)
    for prec in (FP32, BF16):
        Bl = oracle.sketch_apply_lowp(prec, A, s, seed)
        Zr = torch_round(Z, prec)
        exp = (Zr @ A) / math.sqrt(s)
        # exact products of the rounded normals, summed in FP64
        assert np.abs(Bl - exp).max() <= 4 * m * U64 * (np.abs(Zr) @ np.abs(A)).max()
        # and within the normal rounding of the FP64 sketch
        dz = (2.0 ** -24 if prec == FP32 else 2.0 ** -8) * np.abs(Z)
        bound = (dz @ np.abs(A)) / math.sqrt(s) + 4 * m * U64 * np.abs(B64).max()
        assert np.all(np.abs(Bl - B64) <= bound)


def test_sketch_lowp_rounds_the_input():
    """A enters the low-precision sketch as its FP32 rounding for both input types: a column
    of 1 + 2^-30 rounds to all ones, while a column of 1 + 2^-12 (which BF16 itself would
    round to one) survives both."""
    m, s, seed = 257, 8, 3
    A = F(np.stack([np.full(m, 1 + 2.0 ** -30), np.full(m, 1 + 2.0 ** -12)], axis=1))
    ones = F(np.ones((m, 1)))
    for prec in (FP32, BF16):
        Bl = oracle.sketch_apply_lowp(prec, A, s, seed)
        Bones = oracle.sketch_apply_lowp(prec, ones, s, seed)
        assert np.array_equal(Bl[:, :1], Bones)
        assert np.allclose(Bl[:, 1:], Bones * (1 + 2.0 ** -12), rtol=1e-14, atol=0)


def test_sketch_lowp_general_input_is_rounded_normals_times_fp32_input():
    """On a general A (no exact representation in either type) the low-precision sketch is
    torch's rounding of the normals (FP32, then BF16 for BF16 inputs) times numpy's FP32
    rounding of A, summed exactly up to FP64 rounding."""
    m, n, s, seed = 700, 6, 12, 21104
    A = gen_matrix(m, n, 1e6, 77)
    Z = oracle.sketch_normals(seed, 0, s, 0, m)
    A32 = A.astype(np.float32).astype(np.float64)
    for prec in (FP32, BF16):
        Bl = oracle.sketch_apply_lowp(prec, A, s, seed)
        Zr = torch_round(Z, prec)
        exp = (Zr @ A32) / math.sqrt(s)
        assert np.abs(Bl - exp).max() <= 4 * m * U64 * (np.abs(Zr) @ np.abs(A32)).max()
        # the BF16 rounding of A itself would move the sketch far outside that bound
        Ab = torch_round(A, BF16)
        assert np.abs(Bl - (Zr @ Ab) / math.sqrt(s)).max() > 1e3 * 4 * m * U64 * np.abs(exp).max()


def test_three_bf16_terms_carry_an_fp32_value_exactly():
    """The split the BF16 sketch relies on: hi = bf16(x), mid = bf16(x - hi), lo =
    bf16(x - hi - mid), each difference taken in FP32, gives hi + mid + lo = x exactly for
    every normal FP32 x (torch's conversions, random values over the working range and the
    values next to BF16 rounding ties)."""
    rng = np.random.default_rng(9)
    x = (rng.standard_normal(200000) * 10.0 ** rng.integers(-25, 25, 200000)).astype(np.float32)
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 1 + 2.0 ** -8 + 2.0 ** -23,
                     1 - 2.0 ** -24, 3.0 * 2.0 ** -20, 65535.0, -65537.0], dtype=np.float32)
    t = torch.from_numpy(np.concatenate([x, ties]))
    hi = t.to(torch.bfloat16).to(torch.float32)
    r1 = t - hi
    mid = r1.to(torch.bfloat16).to(torch.float32)
    r2 = r1 - mid
    lo = r2.to(torch.bfloat16).to(torch.float32)
    assert torch.equal(lo, r2)  # the last term is exact
    total = hi.double() + mid.double() + lo.double()
    assert torch.equal(total, t.double())


# ------------------------------------------------------------------------- apply ----
def test_apply_rinv_lowp_exact_integers_and_triangularity():
    rng = np.random.default_rng(1)
    m, n = 50, 9
    Y = F(rng.integers(-8, 9, size=(m, n)))
    Rfull = F(rng.integers(-8, 9, size=(n, n)))  # lower part must be ignored
    exp = Y @ np.triu(Rfull)
    for prec in (FP32, BF16):
        X = oracle.apply_rinv_lowp(prec, Y, Rfull)
        assert np.array_equal(X, torch_round(exp, prec))


def test_apply_rinv_lowp_rounds_operands_and_result():
    rng = np.random.default_rng(2)
    m, n = 40, 6
    Y = F(rng.standard_normal((m, n)))
    Rv = F(np.triu(rng.standard_normal((n, n))))
    for prec in (FP32, BF16):
        exact = torch_round(Y, prec) @ torch_round(Rv, prec)  # few terms: FP64 sum is exact
        X = oracle.apply_rinv_lowp(prec, Y, Rv)               # to well below the final rounding
        assert np.array_equal(X, torch_round(exact, prec))


# -------------------------------------------------------------------------- gram ----
def test_gram_lowp_exact_and_rounded():
    rng = np.random.default_rng(3)
    X = F(rng.integers(-16, 17, size=(100, 7)))
    for prec in (FP32, BF16):
        assert np.array_equal(oracle.gram_lowp(prec, X), X.T @ X)
    Xr = F(rng.standard_normal((100, 7)))
    for prec in (FP32, BF16):
        Xp = torch_round(Xr, prec)
        W = oracle.gram_lowp(prec, Xr)
        assert np.array_equal(W, W.T)
        assert np.abs(W - Xp.T @ Xp).max() <= 4 * 100 * U64 * (np.abs(Xp).T @ np.abs(Xp)).max()


# ------------------------------------------------------------------------ driver ----
@pytest.mark.parametrize("prec", [FP32, BF16])
@pytest.mark.parametrize("kappa", [1e4, 1e8, 1e12])
def test_mixed_driver_auto_is_a_qr_factorization(prec, kappa):
    m, n, s = 2048, 16, 32
    A = gen_matrix(m, n, kappa, 211104)
    r = oracle.rxr_cholqr_mixed(A, s, 11104, prec=prec, fp64_passes=0)
    assert r["info"] == 0
    assert 1 <= r["passes"] <= 3
    Q, R = r["Q"], r["R"]
    assert np.array_equal(np.tril(R, -1), np.zeros((n, n)))
    assert np.all(np.diag(R) > 0)
    # FP64 accuracy of a Householder QR, with the same constants as the FP64 method's pins
    assert oracle.orthogonality(Q) <= 2 * math.sqrt(n) * 64 * U64 * n
    assert oracle.residual(A, Q, R) <= 64 * U64 * math.sqrt(n)
    # R is the unique positive-diagonal R factor of A: LAPACK's, to kappa * u
    Rl = signfix(np.linalg.qr(A, mode="r"))
    assert np.linalg.norm(R - Rl) / np.linalg.norm(Rl) <= 4 * n * kappa * U64


def test_mixed_driver_pass_counts():
    """A well-conditioned input needs a single FP64 pass in automatic mode; a fixed count
    is obeyed; BF16 at kappa 1e12 needs more passes than FP32 at kappa 1e4."""
    A4 = gen_matrix(2048, 16, 1e4, 7)
    A12 = gen_matrix(2048, 16, 1e12, 7)
    assert oracle.rxr_cholqr_mixed(A4, 32, 1, prec=FP32, fp64_passes=0)["passes"] == 1
    for k in (1, 2, 3):
        assert oracle.rxr_cholqr_mixed(A4, 32, 1, prec=FP32, fp64_passes=k)["passes"] == k
    assert oracle.rxr_cholqr_mixed(A12, 32, 1, prec=BF16, fp64_passes=0)["passes"] >= 2


def test_mixed_driver_low_precision_breakdown_falls_back():
    """Two columns an FP32 number apart by a factor 1 + 2^-30 (distinct in FP64, equal in
    FP32): the stage's A R0^-1 in FP32 is then far from orthonormal and, for this seeded
    input with the BF16 sketch's R0, its Cholesky breaks down at column 6; R0 alone
    preconditions, and the FP64 passes still give an orthonormal Q.  (Whether the stage
    breaks down depends on R0, so on the sketch: with the FP32 sketch's R0 it does not, and
    the three passes succeed as well.  A fixed pass count always runs the stage; the
    automatic mode would skip it for this cond(R0).)"""
    A = gen_matrix(4096, 32, 1e3, 5)
    A[:, 4] = torch_round(A[:, 4], FP32)
    A[:, 5] = A[:, 4] * (1 + 2.0 ** -30)
    assert np.array_equal(torch_round(A[:, 5], FP32), A[:, 4])
    assert not np.array_equal(A[:, 5], A[:, 4])
    for prec, lp in ((BF16, 6), (FP32, 0)):
        r = oracle.rxr_cholqr_mixed(F(A), 64, 7, prec=prec, fp64_passes=3)
        assert r["lp_info"] == lp
        assert r["info"] == 0 and r["passes"] == 3
        assert oracle.orthogonality(r["Q"]) <= 1e-13


@pytest.mark.parametrize("prec,kappa,runs", [(FP32, 1e4, True), (FP32, 1e10, False),
                                             (BF16, 1e4, True), (BF16, 1e10, False)])
def test_mixed_driver_auto_stage_rule(prec, kappa, runs):
    """Automatic mode runs the low-precision stage iff ||R0||_F ||R0^-1||_F u_p <= 1, with
    u_p = 2^-24 for either sketch type (the stage takes FP32 inputs in both).
    Checked on inputs far from the threshold against LAPACK's R factor of A itself (the
    sketch changes the singular values of R0 by a modest factor only): >= 10x below it the
    stage runs (lp_info 0), >= 10x above it it is skipped (lp_info -1); the result is a
    QR factorization either way."""
    m, n, s = 2048, 16, 32
    A = gen_matrix(m, n, kappa, 311104)
    Rl = np.linalg.qr(A, mode="r")
    est = np.linalg.norm(Rl) * np.linalg.norm(np.linalg.inv(Rl)) * 2.0 ** -24
    assert (est <= 0.1) if runs else (est >= 10.0)
    r = oracle.rxr_cholqr_mixed(A, s, 11104, prec=prec, fp64_passes=0)
    assert r["info"] == 0
    assert r["lp_info"] == (0 if runs else -1)
    assert oracle.orthogonality(r["Q"]) <= 1e-13
    if runs:
        assert r["passes"] == 1


def test_mixed_driver_fixed_single_pass_fails_loudly_or_not_at_all():
    """With one fixed pass and a far too ill-conditioned input the method either succeeds
    or reports a breakdown (stage 3) with NaN outputs; never a silent non-orthogonal Q
    with info 0 beyond the CholeskyQR bound kappa(A1)^2 u."""
    A = gen_matrix(2048, 16, 1e16, 9)
    r = oracle.rxr_cholqr_mixed(A, 32, 1, prec=BF16, fp64_passes=1)
    if r["info"]:
        assert r["info"] // 1000 == 3
        assert np.isnan(r["Q"]).all() and np.isnan(r["R"]).all()
    else:
        assert np.isfinite(r["Q"]).all()
