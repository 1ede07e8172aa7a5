"""Pins of the CPU oracle against things other than itself.

Each test checks one oracle routine against an independent implementation (NumPy,
SciPy/LAPACK, mpmath), a closed form, an invariant, brute force on tiny inputs, or a
bound the paper states.  A plausible mistake in the oracle (dropped term, wrong sign or
index, transposed operand) fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

import oracle
from inputs import sigma_logspaced, gen_matrix, gen_ternary
from paper_claims import paper_claims

U64 = 2.0 ** -53  # unit roundoff
EPS = 2.0 ** -52  # the paper's u (Section 4.1)



def F(x):
    return np.asfortranarray(x, dtype=np.float64)


def signfix(Rm):
    d = np.sign(np.diag(Rm))
    d[d == 0] = 1
    return d[:, None] * Rm


# ------------------------------------------------------------------------------ RNG --
def _numpy_philox_words(ctr, key):
    """Philox4x64-10 via NumPy's independent implementation.  NumPy increments its
    256-bit counter before each block, so seed it with ctr - 1."""
    c = sum(int(x) << (64 * i) for i, x in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    cm1 = np.array([(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=cm1, key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4).astype(np.uint64)


@pytest.mark.parametrize("trial", range(8))
def test_philox4x64_matches_numpy(trial):
    rng = np.random.default_rng(1234 + trial)
    key = rng.integers(0, 2**64, size=2, dtype=np.uint64, endpoint=False)
    ctr = rng.integers(0, 2**64, size=4, dtype=np.uint64, endpoint=False)
    if trial == 0:
        key[:] = 0
        ctr[:] = [1, 0, 0, 0]
    got = oracle.philox4x64_10(ctr, key)
    exp = _numpy_philox_words(ctr, key)
    assert np.array_equal(got, exp)


def test_philox_weyl_constants_from_definition():
    """The key bumps of Philox are fixed-point values of the golden ratio and of
    sqrt(3)-1 (Salmon et al.).  The 64-bit constants are exercised by the NumPy
    cross-check above; the 32-bit ones must be the same irrationals in 32 bits."""
    golden = (math.sqrt(5.0) - 1.0) / 2.0
    assert int(golden * 2**32) == 0x9E3779B9
    assert int((math.sqrt(3.0) - 1.0) * 2**32) == 0xBB67AE85
    # and the key schedule is live: different keys give different words
    assert not np.array_equal(oracle.philox4x32_10([0, 0, 0, 0], [0, 0]),
                              oracle.philox4x32_10([0, 0, 0, 0], [0x9E3779B9, 0xBB67AE85]))


def test_philox4x32_counter_sensitivity():
    """Every input word and every key word changes the output (no dropped input)."""
    base = oracle.philox4x32_10([5, 6, 7, 8], [9, 10])
    for pos in range(4):
        c = [5, 6, 7, 8]
        c[pos] ^= 1
        assert not np.array_equal(oracle.philox4x32_10(c, [9, 10]), base)
    for pos in range(2):
        k = [9, 10]
        k[pos] ^= 1
        assert not np.array_equal(oracle.philox4x32_10([5, 6, 7, 8], k), base)


def test_philox4x32_bits_uniform():
    """Output words are uniform bits: each of the 32 bit positions is set with frequency
    1/2 within 5 standard errors over 2^14 counters."""
    words = np.array([oracle.philox4x32_10([i, 0, 3, 0], [77, 1]) for i in range(4096)])
    bits = ((words.reshape(-1, 1) >> np.arange(32, dtype=np.uint32)) & 1).astype(float)
    freq = bits.mean(axis=0)
    se = 0.5 / math.sqrt(bits.shape[0])
    assert np.all(np.abs(freq - 0.5) < 5 * se)


def test_sketch_normals_distribution():
    """Entries of Z are N(0,1): KS test, moments, and no correlation between the two
    members of a Box-Muller pair or between neighbouring rows."""
    Z = oracle.sketch_normals(11101, 0, 64, 0, 4096)  # 2^18 samples
    z = Z.ravel()
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)
    assert abs(scipy.stats.skew(z)) < 0.03
    assert abs(scipy.stats.kurtosis(z)) < 0.05
    assert scipy.stats.kstest(z, "norm").pvalue > 1e-3
    # pair members (columns 4p and 4p+1 share one Philox call)
    a, b = Z[:, 0::4].ravel(), Z[:, 1::4].ravel()
    assert abs(np.corrcoef(a, b)[0, 1]) < 5 / math.sqrt(a.size)
    c, d = Z[0::2].ravel(), Z[1::2].ravel()
    assert abs(np.corrcoef(c, d)[0, 1]) < 5 / math.sqrt(c.size)
    # different seeds give different streams
    Z2 = oracle.sketch_normals(11102, 0, 64, 0, 64)
    assert not np.allclose(Z2, Z[:, :64])


def test_sketch_normal_block_consistency():
    """Block extraction agrees with single-entry evaluation (index mapping)."""
    Z = oracle.sketch_normals(7, 3, 5, 10, 9)
    for a in range(5):
        for b in range(9):
            assert Z[a, b] == oracle.sketch_normal(7, 3 + a, 10 + b)


# --------------------------------------------------------------------------- sketch --
@pytest.mark.parametrize("m,n,s", [(257, 5, 7), (1000, 16, 32), (64, 1, 1)])
def test_sketch_apply_equals_matmul(m, n, s):
    """B = (Z/sqrt(s)) A, with Z from the oracle's generator and the product by NumPy."""
    A = gen_matrix(m, n, 1e3, 5) if m >= n else None
    Z = oracle.sketch_normals(99, 0, s, 0, m)
    B = oracle.sketch_apply(A, s, 99)
    Bref = (Z / math.sqrt(s)) @ A
    scale = (np.abs(Z) / math.sqrt(s)) @ np.abs(A)
    assert np.all(np.abs(B - Bref) <= 4 * m * U64 * scale + 1e-300)


def test_sketch_apply_leading_dimension_and_linearity():
    A = gen_matrix(300, 6, 1e2, 8)
    buf = np.full((311, 6), np.nan, order="F")
    buf[:300] = A
    Bv = oracle._load  # noqa: F841  (ensure loaded)
    B1 = oracle.sketch_apply(A, 12, 3)
    # a view with lda=311: use the C entry point through a sliced Fortran buffer
    import ctypes

    out = np.zeros((12, 6), order="F")
    oracle._load().or_sketch_apply(300, 6, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   311, 12, 3,
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 12)
    assert np.array_equal(out, B1)
    B2 = oracle.sketch_apply(F(2.0 * A), 12, 3)
    assert np.array_equal(B2, 2.0 * B1)  # scaling by 2 is exact


# ------------------------------------------------------------------ householder QR --
@pytest.mark.parametrize("s,n,kappa", [(64, 32, 1e3), (40, 40, 10.0), (100, 7, 1e8), (9, 1, 1.0)])
def test_householder_matches_lapack(s, n, kappa):
    B = gen_matrix(s, n, kappa, 17)
    R, info = oracle.householder_r(B)
    assert info == 0
    Rl = signfix(np.linalg.qr(B, mode="r"))
    assert np.all(np.diag(R) > 0)
    assert np.all(np.tril(R, -1) == 0)
    err = np.linalg.norm(R - Rl) / np.linalg.norm(Rl)
    assert err < 50 * n * EPS * kappa
    # R^T R = B^T B to backward-error accuracy
    assert np.linalg.norm(R.T @ R - B.T @ B) <= 50 * s * n * EPS * np.linalg.norm(B) ** 2


def test_householder_closed_form_triangular():
    """B = [T; 0] with T upper and positive diagonal has R = T."""
    rng = np.random.default_rng(3)
    T = np.triu(rng.standard_normal((6, 6)))
    np.fill_diagonal(T, np.abs(np.diag(T)) + 0.5)
    B = F(np.vstack([T, np.zeros((10, 6))]))
    R, info = oracle.householder_r(B)
    assert info == 0
    assert np.allclose(R, T, rtol=0, atol=1e-14)
    # negative diagonal entries are flipped row-wise by the sign normalisation
    T2 = T.copy()
    T2[2] *= -1
    R2, _ = oracle.householder_r(F(np.vstack([T2, np.zeros((3, 6))])))
    assert np.allclose(R2, T, rtol=0, atol=1e-14)


def test_householder_rank_deficient_info():
    B = gen_matrix(20, 5, 10.0, 2)
    B[:, 3] = 0.0
    _, info = oracle.householder_r(B)
    assert info == 1004
    B2 = gen_matrix(20, 5, 10.0, 2)
    B2[4, 2] = np.nan
    _, info2 = oracle.householder_r(B2)
    assert info2 != 0


# ----------------------------------------------------------------------------- LU --
@pytest.mark.parametrize("s,n", [(64, 32), (20, 20), (50, 3)])
def test_lu_matches_scipy(s, n):
    B = gen_matrix(s, n, 1e4, 23)
    R, piv, info = oracle.lu_r(B)
    assert info == 0
    lu, ipiv = scipy.linalg.lu_factor(B)  # LAPACK dgetrf (partial pivoting, first max)
    U = np.triu(lu[:n, :n])
    assert np.array_equal(piv, ipiv[:n])
    d = np.sign(np.diag(U))
    assert np.allclose(R, d[:, None] * U, rtol=0, atol=1e-12 * np.abs(U).max())
    assert np.all(np.diag(R) > 0)


def test_lu_tie_break_first_max():
    """Equal magnitudes in the pivot column: the first row wins (LAPACK idamax rule)."""
    B = F([[1.0, 2.0], [-1.0, 5.0], [1.0, 7.0]])
    R, piv, info = oracle.lu_r(B)
    assert info == 0 and piv[0] == 0
    lu, ipiv = scipy.linalg.lu_factor(B)
    assert ipiv[0] == 0


@pytest.mark.parametrize("s,n,seed", [(128, 64, 1), (256, 128, 2), (200, 100, 5)])
def test_lu_ties_at_later_steps_match_lapack(s, n, seed):
    """Entries from {-1, 0, 1}: several steps, after earlier interchanges, see equal
    magnitudes in the pivot column.  The oracle's whole pivot sequence equals LAPACK's
    (first maximum in the current row order), and U agrees to rounding."""
    B = gen_ternary(s, n, seed)
    R, piv, info = oracle.lu_r(B)
    assert info == 0
    lu, ipiv = scipy.linalg.lu_factor(B)
    assert np.array_equal(piv, ipiv[:n])
    U = np.triu(lu[:n, :n])
    d = np.sign(np.diag(U))
    assert np.allclose(R, d[:, None] * U, rtol=0, atol=1e-13 * np.abs(U).max())


def test_lu_zero_pivot_info():
    B = F(np.zeros((6, 3)))
    B[:, 0] = 1.0
    B[:, 1] = 2.0  # column 2 is a multiple of column 1 -> zero pivot at column 2
    B[:, 2] = np.arange(6)
    _, _, info = oracle.lu_r(B)
    assert info == 1002


# ----------------------------------------------------------------------- Cholesky --
@pytest.mark.parametrize("n", [1, 2, 17, 64])
def test_cholesky_matches_numpy(n):
    X = gen_matrix(3 * n + 5, n, 100.0, n)
    W = F(X.T @ X)
    R, info = oracle.cholesky_upper(W)
    assert info == 0
    Rl = np.linalg.cholesky(W).T
    assert np.allclose(R, Rl, rtol=0, atol=100 * n * EPS * np.abs(Rl).max())
    assert np.all(np.tril(R, -1) == 0)


def test_cholesky_reads_upper_only_and_reports_breakdown():
    W = np.eye(4)
    W[2, 2] = -1.0
    W = F(W)
    R, info = oracle.cholesky_upper(W)
    assert info == 3
    assert np.all(np.isnan(R[:3, 2])) and np.all(np.isnan(R[:, 3]))
    assert np.array_equal(R[:2, :2], np.eye(2))
    Wg = F(np.array([[4.0, 2.0], [999.0, 5.0]]))  # lower garbage must be ignored
    R2, info2 = oracle.cholesky_upper(Wg)
    assert info2 == 0
    assert np.allclose(R2, [[2.0, 1.0], [0.0, 2.0]])


# -------------------------------------------------------------------- TRSM / Gram --
def test_trsm_matches_scipy_and_backward_error():
    Y = gen_matrix(500, 24, 1e2, 1)
    T = np.triu(np.random.default_rng(0).standard_normal((24, 24)))
    np.fill_diagonal(T, np.abs(np.diag(T)) + 1.0)
    T = F(T)
    X = oracle.trsm_ru(Y, T)
    Xs = scipy.linalg.solve_triangular(T, Y.T, trans="T", lower=False).T
    assert np.allclose(X, Xs, rtol=1e-12, atol=1e-14)
    # row-wise backward error |Y - X T| <= c n u |X||T|
    assert np.all(np.abs(Y - X @ T) <= 4 * 24 * U64 * (np.abs(X) @ np.abs(T)) + 1e-300)


def test_gram_and_trmm_match_numpy():
    X = gen_matrix(700, 9, 1e3, 4)
    W = oracle.gram(X)
    assert np.allclose(W, X.T @ X, rtol=0, atol=1e-13)
    assert np.array_equal(W, W.T)
    rng = np.random.default_rng(9)
    A = F(np.triu(rng.standard_normal((7, 7))))
    B = F(np.triu(rng.standard_normal((7, 7))))
    C = oracle.trmm_upper(A, B)
    assert np.allclose(C, A @ B, rtol=0, atol=1e-14)
    assert np.all(np.tril(C, -1) == 0)


# ------------------------------------------------------------------------ metrics --
def test_metrics_closed_forms():
    d = 1e-3
    Q = np.zeros((5, 2))
    Q[0, 0] = 1.0
    Q[1, 1] = 1.0
    Q[0, 1] = d  # Q^T Q - I = [[0, d], [d, d^2]]
    assert math.isclose(oracle.orthogonality(F(Q)), math.sqrt(2 * d * d + d ** 4), rel_tol=1e-14)
    P = F(np.eye(7)[:, [3, 0, 5]])
    assert oracle.orthogonality(P) == 0.0
    A = F(np.arange(12.0).reshape(4, 3) + 1.0)
    R = F(np.triu(np.ones((3, 3))))
    Qx = F(np.linalg.solve(R.T, A.T).T)
    res = oracle.residual(A, Qx, R)
    assert res < 1e-15
    A2 = A.copy()
    A2[1, 1] += 1e-6
    assert math.isclose(oracle.residual(F(A2), F(A), F(np.eye(3))), 1e-6 / np.linalg.norm(A2), rel_tol=1e-9)


def test_metrics_against_mpmath():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 4)))
    Q = F(Q)
    E = [[mp.mpf(0)] * 4 for _ in range(4)]
    for a in range(4):
        for b in range(4):
            acc = mp.mpf(0)
            for j in range(40):
                acc += mp.mpf(Q[j, a]) * mp.mpf(Q[j, b])
            E[a][b] = acc - (1 if a == b else 0)
    ref = float(mp.sqrt(sum(E[a][b] ** 2 for a in range(4) for b in range(4))))
    got = oracle.orthogonality(Q)
    assert abs(got - ref) <= 1e-6 * ref


# ------------------------------------------------------------------------ drivers --
def _brute_force_qr(A):
    """Textbook Householder QR written independently (no pivoting), sign-normalised."""
    m, n = A.shape
    Rw = A.astype(np.float64).copy()
    Qf = np.eye(m)
    for k in range(n):
        x = Rw[k:, k].copy()
        e = np.zeros_like(x)
        e[0] = np.linalg.norm(x) * (1.0 if x[0] < 0 else -1.0)
        v = x - e
        nv = np.linalg.norm(v)
        if nv == 0:
            continue
        v /= nv
        Rw[k:, :] -= 2.0 * np.outer(v, v @ Rw[k:, :])
        Qf[:, k:] -= 2.0 * np.outer(Qf[:, k:] @ v, v)
    R = np.triu(Rw[:n])
    Q = Qf[:, :n]
    d = np.sign(np.diag(R))
    return Q * d[None, :], d[:, None] * R


@pytest.mark.parametrize("variant", [oracle.RQR, oracle.RLU])
@pytest.mark.parametrize("m,n,kappa", [(64, 8, 1e3), (48, 5, 10.0), (33, 3, 1e2)])
def test_driver_matches_brute_force_householder(variant, m, n, kappa):
    """P1: on tiny inputs the result is the unique thin QR with positive diag(R)."""
    A = gen_matrix(m, n, kappa, 41)
    r = oracle.rxr_cholqr(A, 2 * n, 7, variant=variant)
    assert r["info"] == 0
    Qb, Rb = _brute_force_qr(A)
    tol = 100 * n * EPS * kappa
    assert np.linalg.norm(r["R"] - Rb) / np.linalg.norm(Rb) < tol
    assert np.linalg.norm(r["Q"] - Qb) < tol * math.sqrt(n)
    assert np.all(np.diag(r["R"]) > 0)
    assert np.all(np.tril(r["R"], -1) == 0)


def test_driver_closed_forms():
    """P2: kappa = 1 gives R = I, Q = A; n = 1 gives R = ||a||; [T; 0] gives R = T."""
    A = gen_matrix(200, 6, 1.0, 3)  # = U V^T, orthonormal columns
    r = oracle.rxr_cholqr(A, 12, 1)
    assert np.allclose(r["R"], np.eye(6), rtol=0, atol=1e-14)
    assert np.allclose(r["Q"], A, rtol=0, atol=1e-14)
    a = F(np.random.default_rng(1).standard_normal((100, 1)))
    r1 = oracle.rxr_cholqr(a, 2, 5)
    nrm = np.linalg.norm(a)
    assert math.isclose(r1["R"][0, 0], nrm, rel_tol=1e-14)
    assert np.allclose(r1["Q"][:, 0], a[:, 0] / nrm, rtol=0, atol=1e-15)
    rng = np.random.default_rng(2)
    T = np.triu(rng.standard_normal((4, 4)))
    np.fill_diagonal(T, np.abs(np.diag(T)) + 1.0)
    A3 = F(np.vstack([T, np.zeros((60, 4))]))
    r3 = oracle.rxr_cholqr(A3, 8, 2)
    assert np.allclose(r3["R"], T, rtol=0, atol=1e-13)
    assert np.allclose(r3["Q"], np.eye(64, 4), rtol=0, atol=1e-13)


def test_driver_invariances():
    """P4: column scaling (Q, R D); row permutation (Pi Q, R); rQR and rLU agree."""
    A = gen_matrix(512, 10, 1e6, 12)
    base = oracle.rxr_cholqr(A, 20, 3)
    Dg = np.array([1.0, 2.0, 0.5, 3.0, 7.0, 1e-3, 1.0, 4.0, 0.25, 10.0])
    sc = oracle.rxr_cholqr(F(A * Dg[None, :]), 20, 3)
    tol = 1e3 * EPS * 1e6
    assert np.linalg.norm(sc["R"] - base["R"] * Dg[None, :]) / np.linalg.norm(sc["R"]) < tol
    assert np.linalg.norm(sc["Q"] - base["Q"]) < tol
    perm = np.random.default_rng(0).permutation(512)
    pr = oracle.rxr_cholqr(F(A[perm]), 20, 3)
    assert np.linalg.norm(pr["R"] - base["R"]) / np.linalg.norm(base["R"]) < tol
    assert np.linalg.norm(pr["Q"] - base["Q"][perm]) < tol
    lu = oracle.rxr_cholqr(A, 20, 3, variant=oracle.RLU)
    assert np.linalg.norm(lu["R"] - base["R"]) / np.linalg.norm(base["R"]) < tol


def test_preconditioning_identity_prop():
    """P5 (Section 3, Proposition on cond(X) = cond(PQ)): cond(A R0^{-1}) equals
    cond(S Q_A), with S regenerated from the seed and Q_A from LAPACK."""
    for kappa in (1e2, 1e6):
        A = gen_matrix(300, 12, kappa, 77)
        s = 24
        r = oracle.rxr_cholqr(A, s, 555)
        A1 = oracle.trsm_ru(A, r["R0"])
        S = oracle.sketch_normals(555, 0, s, 0, 300) / math.sqrt(s)
        QA, _ = np.linalg.qr(A)
        c1, c2 = np.linalg.cond(A1), np.linalg.cond(S @ QA)
        assert abs(c1 - c2) / c2 < 1e3 * EPS * kappa


def test_gaussian_theorem_and_marchenko_pastur():
    """P6 (Section 3, Gaussian Ensemble theorem): at l = 2n the preconditioned matrix
    obeys the theorem's bound, and cond(A1) is distributed like the condition number of
    an l x n Gaussian matrix (by the Proposition of Section 3), whose mean sits near the
    Marchenko-Pastur edge ratio (1+sqrt(n/l))/(1-sqrt(n/l))."""
    c = paper_claims()
    n, s, m = 64, 128, 1024
    bound = (c["gaussian_bound_numer"] + math.sqrt(n / s)) / (1 - math.sqrt(n / s))
    conds = []
    for k in range(12):
        A = gen_matrix(m, n, 1e8, 900 + k)
        r = oracle.rxr_cholqr(A, s, 31 + k)
        conds.append(np.linalg.cond(oracle.trsm_ru(A, r["R0"])))
    conds = np.array(conds)
    assert np.all(conds <= bound)
    rng = np.random.default_rng(0)
    gauss = np.array([np.linalg.cond(rng.standard_normal((s, n))) for _ in range(200)])
    # same distribution: two-sample KS and means within 4 standard errors
    assert scipy.stats.ks_2samp(conds, gauss).pvalue > 1e-3
    se = gauss.std() * math.sqrt(1 / len(conds) + 1 / len(gauss))
    assert abs(conds.mean() - gauss.mean()) < 4 * se
    mp_edge = (1 + math.sqrt(n / s)) / (1 - math.sqrt(n / s))
    assert abs(conds.mean() - mp_edge) / mp_edge < 0.15


def test_sampling_rate_study():
    """P7 (Section 4.5): l/n = 1.2 brings cond(A1) to about 20 and larger ratios keep
    shrinking it; l = n gives much larger values."""
    c = paper_claims()
    n, m = 64, 1024
    means = {}
    for ratio in (1.0, c["sampling_ratio_small"], c["sampling_recommended_lo"],
                  c["sampling_recommended_hi"]):
        s = int(round(ratio * n))
        vals = []
        for k in range(6):
            A = gen_matrix(m, n, 1e6, 300 + k)
            r = oracle.rxr_cholqr(A, s, 70 + k)
            vals.append(np.linalg.cond(oracle.trsm_ru(A, r["R0"])))
        means[ratio] = float(np.median(vals))
    assert means[1.0] > 100
    assert 8 < means[c["sampling_ratio_small"]] < 3 * c["sampling_cond_small"]
    assert means[1.5] < means[c["sampling_ratio_small"]] and means[2.0] < means[1.5]
    assert means[2.0] < 8


def test_cholqr_kappa_laws():
    """P10 (Section 2.1 and Section 4.2): plain CholeskyQR loses orthogonality like
    kappa^2 u and breaks down past kappa ~ 1e8; CholeskyQR2 too; the preconditioned
    method's orthogonality does not depend on kappa."""
    c = paper_claims()
    u = c["u"]
    for kappa in (1e3, 1e5, 1e7):
        A = gen_matrix(2048, 16, kappa, 5)
        Q, R, info = oracle.cholqr_n(A, 1)
        assert info == 0
        o = oracle.orthogonality(Q)
        assert 1e-3 * kappa ** 2 * u < o < 1e2 * kappa ** 2 * u
    for kappa in (1e10, 1e12):
        # breakdown (or useless output) in at least two of three matrices
        fail1 = fail2 = 0
        for seed in (5, 6, 7):
            A = gen_matrix(4096, 16, kappa, seed)
            Q, R, info = oracle.cholqr_n(A, 1)
            fail1 += info != 0 or oracle.orthogonality(Q) > 0.1
            Q2, R2, info2 = oracle.cholqr_n(A, 2)
            fail2 += info2 != 0 or oracle.orthogonality(Q2) > 1e-6
        assert fail1 >= 2 and fail2 >= 2
    orths = []
    for kappa in (1e3, 1e8, 1e12, 1e15):
        A = gen_matrix(2048, 16, kappa, 5)
        r = oracle.rxr_cholqr(A, 32, 9, extra_pass=False)
        assert r["info"] == 0
        orths.append(oracle.orthogonality(r["Q"]))
    assert max(orths) < 1e-13


def test_cholqr2_bound_on_extra_pass():
    """P11 (Section 2.1): the extra CholeskyQR pass meets ||Q^T Q - I||_F <=
    6 (m + n + 1) n u, and the residual stays at the u level for every kappa."""
    c = paper_claims()
    m, n = 4096, 32
    for kappa in (1e4, 1e10, 1e14):
        A = gen_matrix(m, n, kappa, 211101)
        for variant in (oracle.RQR, oracle.RLU):
            r = oracle.rxr_cholqr(A, 2 * n, 11101, variant=variant)
            assert r["info"] == 0
            o = oracle.orthogonality(r["Q"])
            assert o <= c["cholqr2_bound_c"] * (m + n + 1) * n * c["u"]
            assert oracle.residual(A, r["Q"], r["R"]) < 1e-14


def test_shifted_cholqr3_survives_high_kappa():
    """sCholeskyQR3 (Section 2.1, shift of Section 4.1's choice) works where CQR2 fails."""
    A = gen_matrix(2048, 16, 1e12, 6)
    Q, R, info = oracle.cholqr_n(A, 3, shift=1e-15 * 1.0)
    assert info == 0
    assert oracle.orthogonality(Q) < 1e-13
    assert oracle.residual(A, Q, R) < 1e-14


def test_driver_breakdown_info_and_nan():
    A = gen_matrix(256, 8, 1e3, 1)
    A[:, 5] = A[:, 2]  # exactly rank deficient
    r = oracle.rxr_cholqr(A, 16, 1)
    if r["info"] != 0:
        assert r["info"] // 1000 in (1, 2, 3)
        assert np.all(np.isnan(r["Q"])) and np.all(np.isnan(r["R"]))
    else:
        # rounding kept every pivot nonzero: the rank deficiency then shows in R's
        # diagonal, and the output is still a valid (non-unique) QR of A
        d = np.abs(np.diag(r["R"]))
        assert d.min() < 1e-14 * d.max()
        assert oracle.orthogonality(r["Q"]) < 1e-13
        assert oracle.residual(A, r["Q"], r["R"]) < 1e-14
    A2 = gen_matrix(256, 8, 1e3, 1)
    A2[:, 4] = 0.0
    r2 = oracle.rxr_cholqr(A2, 16, 1)
    assert r2["info"] == 1005


def test_split_rows_partials_sum_to_whole():
    """Row-partitioned evaluation (one device per row block) reproduces the sketch and
    the Gram matrices: sum of per-block partials equals the whole up to rounding."""
    A = gen_matrix(1200, 10, 1e4, 3)
    Bfull = oracle.sketch_apply(A, 20, 4)
    # block j-range sketches: columns of S indexed by the global row
    parts = []
    for lo, hi in ((0, 400), (400, 1000), (1000, 1200)):
        Z = oracle.sketch_normals(4, 0, 20, lo, hi - lo) / math.sqrt(20)
        parts.append(Z @ A[lo:hi])
    assert np.allclose(sum(parts), Bfull, rtol=0, atol=1e-12)
    W = oracle.gram(A)
    Wp = sum(oracle.gram(F(A[lo:hi])) for lo, hi in ((0, 400), (400, 1000), (1000, 1200)))
    assert np.allclose(W, Wp, rtol=0, atol=1e-13)


def test_sigma_logspaced_definition():
    s = sigma_logspaced(5, 1e4)
    assert np.allclose(s, [1.0, 1e-1, 1e-2, 1e-3, 1e-4], rtol=1e-14)
    A = gen_matrix(100, 5, 1e4, 0)
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(sv, s, rtol=1e-10)
