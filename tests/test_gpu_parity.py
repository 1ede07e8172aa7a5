"""GPU parity: every step of the HIP path against the FP64 CPU oracle, through the C ABI.

Inputs come from the seeded generator (inputs/) only; expected values come from the
oracle only.  Tolerances are derived from the arithmetic of each step (see the
docstrings) and are written into each test.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2111_11148_amd as tsqr
from inputs import gen_matrix, gen_ternary
from gpu_helpers import gpu_orthogonality, gpu_residual, host, rel_fro
from sketch_bounds import fp64_sketch_tol

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
EPS = 2.0 ** -52

# Absolute error bound of one device normal: the device evaluates Box-Muller in FP32 with
# the hardware log2 / sqrt / sin / cos (each within a few FP32 ulps), so an entry of
# magnitude up to 6 carries at most ~16 ulp(FP32) of 6 = 6e-6; the bound adds margin.
NORMAL_ABS_TOL = 2e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    tsqr.load()
    torch.cuda.synchronize()
    yield


def dev(A, ld=None):
    return tsqr.to_device_colmajor(A, ld=ld)


# ------------------------------------------------------------------------ generator --
def test_philox_words_bit_exact():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:4] = [[0, 0, 0, 0], [1, 0, 0, 0], [0xFFFFFFFF] * 4, [5, 6, 7, 8]]
    for seed in (0, 11102, 0xDEADBEEF12345678):
        got = tsqr.philox4x32_10(torch.from_numpy(ctr.view(np.int32)).cuda(), seed)
        got = got.cpu().numpy().view(np.uint32)
        key = [seed & 0xFFFFFFFF, seed >> 32]
        exp = np.array([oracle.philox4x32_10(c, key) for c in ctr])
        assert np.array_equal(got, exp)


@pytest.mark.parametrize("i0,ni,j0,nj", [(0, 64, 0, 4096), (13, 7, 2**20 - 5, 37),
                                         (0, 3, 2**33, 8)])
def test_sketch_normals_match_oracle(i0, ni, j0, nj):
    seed = 11101
    Zg = host(tsqr.sketch_normals(seed, i0, ni, j0, nj))
    Zo = oracle.sketch_normals(seed, i0, ni, j0, nj)
    err = np.abs(Zg - Zo)
    print(f"max |z_gpu - z_oracle| = {err.max():.3e}")
    assert np.all(err <= NORMAL_ABS_TOL)
    # the FP32 entries are exact in FP64
    assert np.array_equal(Zg, Zg.astype(np.float32).astype(np.float64))


# ---------------------------------------------------------------------------- sketch --
@pytest.mark.parametrize("m,n,s", [(5000, 16, 8192), (3001, 40, 2500),
                                   (4096, 32, 64), (1000, 5, 7), (1027, 17, 40), (3000, 128, 256),
                                   (777, 1, 1), (2050, 100, 100), (513, 64, 129), (4100, 200, 400),
                                   (2000, 600, 1200)])
def test_sketch_parity(m, n, s):
    """Against the oracle: |B_gpu - B_or| <= rs (NORMAL_ABS_TOL sum_j |A_jc| +
    4 m u sum_j |z_ij A_jc|), where the first term is the device normals' FP32 evaluation.
    FP64 arithmetic of the product (a property of the device path): B_gpu equals
    rs (Z_dev A) for the normals Z_dev the device generates (read through the normals
    accessor) to within the FP64 summation bound 4 m u |Z_dev||A|, which an FP32 product
    fails by orders of magnitude (tests/test_sketch_bounds.py)."""
    A = gen_matrix(m, n, 1e6, 300 + m)
    seed = 7 + n
    Bg = host(tsqr.sketch(dev(A), s, seed))
    Bo = oracle.sketch_apply(A, s, seed)
    Z = oracle.sketch_normals(seed, 0, s, 0, m)
    rs = 1.0 / math.sqrt(s)
    tol = rs * (NORMAL_ABS_TOL * np.abs(A).sum(axis=0)[None, :] + 4 * m * U * (np.abs(Z) @ np.abs(A)))
    assert np.all(np.abs(Bg - Bo) <= tol)
    Zd = host(tsqr.sketch_normals(seed, 0, s, 0, m))
    ref = rs * (Zd @ A)
    tol64 = fp64_sketch_tol(Zd, A, s, ref)
    err = np.abs(Bg - ref)
    print(f"m={m} n={n} s={s}: max |B - rs Z_dev A| / fp64 bound = {(err / tol64).max():.3e}")
    assert np.all(err <= tol64)


def test_sketch_leading_dimension_and_determinism():
    m, n, s = 2000, 24, 48
    A = gen_matrix(m, n, 1e3, 5)
    B1 = host(tsqr.sketch(dev(A), s, 3))
    B2 = host(tsqr.sketch(dev(A, ld=m + 37), s, 3))
    assert np.array_equal(B1, B2)  # fixed-order reduction, same blocking


# ---------------------------------------------------------------------- small factors --
@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
@pytest.mark.parametrize("s,n,kappa", [(64, 32, 1e4), (256, 128, 1e8), (40, 40, 1e3), (9, 1, 1.0),
                                       (300, 150, 1e5), (512, 256, 1e6), (130, 65, 1e2),
                                       (1000, 100, 1e5), (1536, 700, 1e4), (512, 200, 1e12),
                                       (2048, 1024, 1e8), (700, 333, 1e6),
                                       (3000, 200, 1e6), (8192, 64, 1e4), (4100, 300, 1e8),
                                       (200, 100, 1e10), (256, 65, 1e6), (129, 128, 1e3),
                                       (250, 127, 1e12), (128, 64, 1e8), (256, 50, 1e10),
                                       (500, 60, 1e6)])
def test_sketch_factor_parity(variant, s, n, kappa):
    """R0 is the unique (sign-normalised) R or U factor: ||dR0||/||R0|| <= c n u kappa(B)."""
    B = gen_matrix(s, n, kappa, 17 + s)
    R0g, info = tsqr.sketch_factor(dev(B), variant)
    assert int(info.item()) == 0
    R0g = host(R0g)
    if variant == tsqr.RQR:
        R0o, inf_o = oracle.householder_r(B)
    else:
        R0o, _, inf_o = oracle.lu_r(B)
    assert inf_o == 0
    assert np.all(np.tril(R0g, -1) == 0) and np.all(np.diag(R0g) > 0)
    growth = 1.0 if variant == tsqr.RQR else 10.0
    assert rel_fro(R0g, R0o) <= 50 * n * EPS * kappa * growth


@pytest.mark.parametrize("s,n,seed", [(128, 64, 1), (256, 128, 2), (64, 32, 3), (512, 100, 4),
                                      (200, 100, 5)])
def test_sketch_lu_ties_first_position(s, n, seed):
    """Entries from {-1, 0, 1} keep the eliminated values small integers early on, so
    several steps see distinct rows with equal |a| in the pivot column (4-6 such steps for
    these seeds).  The pivot is the first of them in the current row order, as in the
    oracle's explicit interchanges; another choice would change rows of U by O(1), while
    the same choices leave only rounding (the matrices have cond <= 7)."""
    B = gen_ternary(s, n, seed)
    R0g, info = tsqr.sketch_factor(dev(B), tsqr.RLU)
    R0o, _, inf_o = oracle.lu_r(B)
    assert inf_o == 0 and int(info.item()) == 0
    assert rel_fro(host(R0g), R0o) <= 1e-12


@pytest.mark.parametrize("s,n,seed", [(128, 64, 1), (256, 128, 2), (64, 32, 3), (512, 100, 4),
                                      (200, 100, 5)])
def test_sketch_lu_nan_pivot_reported(s, n, seed):
    """The device takes NaN as the largest pivot candidate (a reading of its own: the
    oracle follows LAPACK's comparison, under which a lone NaN below the diagonal never
    wins).  A NaN in column 5 then always surfaces at step 5: it is the pivot there, or an
    earlier pivot row carried it into every row of column 5.  So every LU kernel class must
    report column 6 (1-based) and put NaN on R0's diagonal there."""
    B = gen_matrix(s, n, 10.0, seed)
    B[s // 3, 5] = np.nan
    R0g, info = tsqr.sketch_factor(dev(B), tsqr.RLU)
    assert int(info.item()) == 1000 + 6
    assert np.isnan(host(R0g)[5, 5])


@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
@pytest.mark.parametrize("s,n", [(128, 64), (256, 128), (64, 32), (512, 100), (3000, 200)])
def test_sketch_factor_nan_diagonal_reported(variant, s, n):
    """A NaN column of the sketch (what a NaN column of A gives) makes that column's
    diagonal entry NaN in either factorization; like the oracle (which flags a zero or NaN
    pivot), every kernel class reports it in info rather than leaving the breakdown to
    a later stage."""
    B = gen_matrix(s, n, 10.0, 7)
    B[:, 9] = np.nan
    R0g, info = tsqr.sketch_factor(dev(B), variant)
    _, inf_o = (oracle.householder_r(B) if variant == tsqr.RQR else oracle.lu_r(B)[::2])
    assert inf_o == 1000 + 10
    assert int(info.item()) == inf_o
    assert np.isnan(host(R0g)[9, 9])


@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
def test_nan_entry_of_a_reported_at_the_sketch_factor(variant):
    """One NaN entry of A fills its column of the sketch with NaN, so the factorization of
    the sketch breaks down at that column: the device reports the oracle's info (stage 1)
    and poisons Q and R."""
    A = gen_matrix(3000, 40, 1e4, 11)
    A[1234, 17] = np.nan
    ref = oracle.rxr_cholqr(A, 80, 5, variant=variant)
    assert ref["info"] == 1000 + 18
    Q, R, info = tsqr.rxr_cholqr(dev(A), 80, 5, variant=variant)
    assert int(info.item()) == ref["info"]
    assert torch.isnan(Q).all() and torch.isnan(R).all()


def test_sketch_factor_breakdown():
    B = gen_matrix(64, 8, 10.0, 1)
    B[:, 3] = 0.0
    for variant in (tsqr.RQR, tsqr.RLU):
        R0, info = tsqr.sketch_factor(dev(B), variant)
        assert int(info.item()) == 1004
        assert np.isnan(host(R0)[3, 3])


@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
@pytest.mark.parametrize("s,n,col", [(512, 200, 100), (1024, 300, 257), (2048, 600, 599),
                                     (256, 128, 70), (130, 65, 64), (200, 100, 31),
                                     (128, 64, 40), (300, 60, 59)])
def test_sketch_factor_breakdown_later_panel(variant, s, n, col):
    """A zero column inside a later panel of the blocked factorizations (or of a later
    row block or column half of the one-column-per-lane QR): the code names that column,
    as the oracle's does, and R0 carries a NaN there."""
    B = gen_matrix(s, n, 10.0, 5 + col)
    B[:, col] = 0.0
    R0, info = tsqr.sketch_factor(dev(B), variant)
    if variant == tsqr.RQR:
        _, inf_o = oracle.householder_r(B)
    else:
        _, _, inf_o = oracle.lu_r(B)
    assert inf_o == 1000 + col + 1
    assert int(info.item()) == inf_o
    assert np.isnan(host(R0)[col, col])


# ---------------------------------------------------------------------------- TRSM ----
@pytest.mark.parametrize("m,n", [(4096, 32), (1000, 5), (1027, 17), (5000, 128), (333, 1),
                                 (2049, 100), (700, 256), (64, 64), (3001, 129), (2000, 200),
                                 (4100, 256), (3000, 1024), (1500, 555)])
def test_trsm_parity(m, n):
    """Row-wise backward error |Y - X T| <= c n u |X||T| (as for the oracle's own solve;
    the column-blocked solve used above 128 columns has the same bound), and X agrees
    with the oracle within c n u cond(T)."""
    Y = gen_matrix(m, n, 1e2, m + n)
    Tm = gen_matrix(3 * n + 8, n, 1e3, n)
    T, _ = oracle.householder_r(Tm)
    Xg = host(tsqr.trsm(dev(Y), dev(T)))
    Xo = oracle.trsm_ru(Y, T)
    back = np.abs(Y - Xg @ T)
    assert np.all(back <= 8 * n * U * (np.abs(Xg) @ np.abs(T)) + 1e-300)
    assert rel_fro(Xg, Xo) <= 10 * n * EPS * 1e3


@pytest.mark.parametrize("n,kappa", [(64, 1e14), (128, 1e14), (128, 1e12), (200, 1e13)])
def test_trsm_ill_conditioned_sketch_factor(n, kappa):
    """T = R0 of the sketch of an ill-conditioned A (as in the first solve of the chain):
    its 16 x 16 diagonal blocks are ill-conditioned, so the solve takes the correction
    step after multiplying by their inverses.  The row-wise backward error stays at the
    substitution's level, |A - X T| <= 8 n u |X||T|, and X = A T^{-1} is well conditioned
    (the preconditioning of the paper's Section 3: cond(X) = cond(S Q_A) = O(1))."""
    m, s = 20000, 2 * n
    A = gen_matrix(m, n, kappa, 900 + n)
    T, info = oracle.householder_r(oracle.sketch_apply(A, s, 31 + n))
    assert info == 0
    Xg = host(tsqr.trsm(dev(A), dev(T)))
    back = np.abs(A - Xg @ T)
    ratio = back / (n * U * (np.abs(Xg) @ np.abs(T)) + 1e-300)
    sv = np.linalg.svd(Xg, compute_uv=False)
    print(f"n={n} kappa={kappa:g}: cond(T)={np.linalg.cond(T):.2e}, max backward error "
          f"/ (n u |X||T|) = {ratio.max():.3f}, cond(X) = {sv[0] / sv[-1]:.2f}")
    assert ratio.max() <= 8
    assert sv[0] / sv[-1] < 50


@pytest.mark.parametrize("n", [64, 200])
def test_trsm_in_place_and_ld(n):
    m = 3000
    Y = gen_matrix(m, n, 10.0, 1)
    T, _ = oracle.householder_r(gen_matrix(3 * n, n, 10.0, 2))
    Yd = dev(Y, ld=m + 5)
    Xo = host(tsqr.trsm(dev(Y), dev(T)))
    tsqr.trsm(Yd, dev(T), X=Yd)
    assert np.array_equal(host(Yd), Xo)


# ---------------------------------------------------------------------------- Gram ----
@pytest.mark.parametrize("m,n", [(4096, 32), (1000, 5), (1027, 17), (6000, 128), (129, 1),
                                 (2049, 100), (1500, 256), (64, 64), (3000, 300), (2000, 1024),
                                 (700, 513)])
def test_gram_parity(m, n):
    """|W_gpu - X^T X| <= 2 m u |X|^T |X| (any summation order), symmetric."""
    X = gen_matrix(m, n, 1e4, 9 + n)
    Wg = host(tsqr.gram(dev(X)))
    Wo = oracle.gram(X)
    assert np.all(np.abs(Wg - Wo) <= 2 * m * U * (np.abs(X).T @ np.abs(X)))
    assert np.array_equal(Wg, Wg.T)


# ------------------------------------------------------------------------ Cholesky ----
@pytest.mark.parametrize("n", [1, 5, 16, 32, 64, 65, 100, 128, 129, 200, 256, 600, 1024])
def test_potrf_parity(n):
    """R^T R = W to c n u ||W||; R agrees with the oracle within c n u cond(W)."""
    X = gen_matrix(4 * n + 10, n, 30.0, n)
    W = np.asfortranarray(X.T @ X)
    Rg, info = tsqr.potrf(dev(W), stage=2)
    assert int(info.item()) == 0
    Rg = host(Rg)
    Ro, io = oracle.cholesky_upper(W)
    assert io == 0
    assert np.all(np.tril(Rg, -1) == 0)
    assert np.linalg.norm(Rg.T @ Rg - W) <= 20 * n * EPS * np.linalg.norm(W)
    assert rel_fro(Rg, Ro) <= 20 * n * EPS * 900.0


@pytest.mark.parametrize("n", [65, 128, 200, 333])
@pytest.mark.parametrize("kappa_w", [1e10, 1e13])
def test_potrf_ill_conditioned(n, kappa_w):
    """The blocked Cholesky is backward stable at any conditioning it completes:
    ||R^T R - W|| <= c n u ||W||, and R within c n u cond(W) of the oracle's factor."""
    X = gen_matrix(4 * n + 10, n, math.sqrt(kappa_w), 7 + n)
    W = np.asfortranarray(X.T @ X)
    Rg, info = tsqr.potrf(dev(W), stage=2)
    assert int(info.item()) == 0
    Rg = host(Rg)
    Ro, io = oracle.cholesky_upper(W)
    assert io == 0
    assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) > 0)
    assert np.linalg.norm(Rg.T @ Rg - W) <= 20 * n * EPS * np.linalg.norm(W)
    assert rel_fro(Rg, Ro) <= 20 * n * EPS * kappa_w


@pytest.mark.parametrize("n", [40, 128, 300])
def test_potrf_in_place_without_workspace(n):
    """R may be W itself (same leading dimension); the call takes no workspace."""
    X = gen_matrix(3 * n + 5, n, 10.0, 11 + n)
    W = np.asfortranarray(X.T @ X)
    Wd = dev(W)
    ref, _ = tsqr.potrf(dev(W), stage=2)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ld = Wd.stride(1)
    rc = tsqr.load().tsqr_potrf(n, Wd.data_ptr(), ld, Wd.data_ptr(), ld, 2, info.data_ptr(),
                                None, 0, None)
    assert rc == 0
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert torch.equal(Wd, ref)


def test_potrf_breakdown_and_upper_only():
    W = np.eye(6)
    W[3, 3] = -1.0
    W[5, 0] = 77.0  # lower garbage is ignored
    R, info = tsqr.potrf(dev(np.asfortranarray(W)), stage=3)
    assert int(info.item()) == 3004
    Rh = host(R)
    assert np.all(np.isnan(Rh[3:, 3:][np.triu_indices(3)]))
    assert np.array_equal(Rh[:3, :3], np.eye(3))


@pytest.mark.parametrize("n", [100, 200])
def test_potrf_breakdown_blocked_panel(n):
    """Breakdown inside a later panel of the blocked factorization (n = 100: one workgroup
    with the matrix in LDS, 16-row panels; n = 200: 32-column panels in place)."""
    W = np.eye(n)
    W[40, 40] = -1.0
    W[n - 50, 3] = 77.0  # lower garbage is ignored
    R, info = tsqr.potrf(dev(np.asfortranarray(W)), stage=3)
    assert int(info.item()) == 3041
    Rh = host(R)
    assert np.all(np.isnan(Rh[40:, 40:][np.triu_indices(n - 40)]))
    assert np.array_equal(Rh[:40, :40], np.eye(40))
    assert np.all(np.tril(Rh, -1) == 0)


@pytest.mark.parametrize("n", [6, 40, 64, 100, 128, 200])
@pytest.mark.parametrize("where", ["diagonal", "off_diagonal"])
def test_potrf_nan_entry_reported(n, where):
    """A NaN in W is a breakdown at the first pivot it reaches (a NaN pivot is not
    positive): a NaN diagonal entry at its own column, an off-diagonal one W(i, j), i < j,
    at column j.  The device names the column the oracle names (its 1-based index plus
    1000 stage)."""
    X = gen_matrix(3 * n + 4, n, 10.0, 31 + n)
    W = np.asfortranarray(X.T @ X)
    j = n - 2 if n < 10 else (2 * n) // 3
    if where == "diagonal":
        W[j, j] = np.nan
    else:
        W[1, j] = W[j, 1] = np.nan
    _, io = oracle.cholesky_upper(W)
    assert io == j + 1
    R, info = tsqr.potrf(dev(W), stage=3)
    assert int(info.item()) == 3000 + j + 1
    Rh = host(R)
    assert np.all(np.isfinite(Rh[:, :j]))
    assert np.isnan(Rh[j, j])


def test_trmm_parity():
    rng = np.random.default_rng(0)
    for n in (1, 7, 32, 128, 200):
        A = np.asfortranarray(np.triu(rng.standard_normal((n, n))))
        B = np.asfortranarray(np.triu(rng.standard_normal((n, n))))
        Cg = host(tsqr.trmm_upper(dev(A), dev(B)))
        Co = oracle.trmm_upper(A, B)
        assert np.all(np.abs(Cg - Co) <= 2 * n * U * (np.abs(A) @ np.abs(B)))


# ---------------------------------------------------------------------- end to end ----
def _check_qr(A, Qd, Rd, Q, R, info, ortho_tol=1e-12, res_tol=1e-13):
    assert int(info) == 0
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    ortho = oracle.orthogonality(Q)
    res = oracle.residual(A, Q, R)
    assert ortho <= ortho_tol, ortho
    assert res <= res_tol, res
    return ortho, res


@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
@pytest.mark.parametrize("m,n,s,kappa", [(4096, 32, 64, 1e10), (4096, 32, 64, 1e14),
                                         (1000, 7, 14, 1e8), (1027, 17, 33, 1e12),
                                         (6000, 128, 256, 1e14), (2500, 100, 200, 1e6),
                                         (64, 64, 128, 1e4), (300, 1, 2, 1.0),
                                         (3000, 256, 512, 1e12), (800, 20, 20, 1e3),
                                         (12000, 48, 4000, 1e10)])
def test_end_to_end_parity(variant, m, n, s, kappa):
    """Q, R of the GPU path: orthogonality <= 1e-12 and residual <= 1e-13 (the targets),
    R upper with positive diagonal, and R within c kappa u of the oracle's R (both are
    backward-stable routes to the unique thin QR; perturbation theory bounds the gap)."""
    A = gen_matrix(m, n, kappa, 211101 + m + n)
    seed = 11101 + n
    Ad = dev(A)
    Qd, Rd, info = tsqr.rxr_cholqr(Ad, s, seed, variant=variant, extra_pass=True)
    Q, R = host(Qd), host(Rd)
    ortho, res = _check_qr(A, Qd, Rd, Q, R, int(info.item()))
    ref = oracle.rxr_cholqr(A, s, seed, variant=variant, extra_pass=True)
    assert ref["info"] == 0
    rd = rel_fro(R, ref["R"])
    print(f"variant={variant} m={m} n={n} s={s} kappa={kappa:g}: ortho={ortho:.2e} "
          f"res={res:.2e} relR={rd:.2e}")
    assert rd <= 100 * n * EPS * kappa + 1e-14
    if kappa <= 1e4:  # well-conditioned: Q agrees elementwise too
        assert np.max(np.abs(Q - ref["Q"])) <= 100 * n * EPS * kappa


@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
@pytest.mark.parametrize("m,n,s,kappa", [(3000, 600, 1200, 1e12), (2100, 1024, 2048, 1e8)])
def test_end_to_end_wide_plain(variant, m, n, s, kappa):
    """The wide configuration's method (no extra pass) at sizes the oracle finishes:
    column-blocked solves, the wide Gram kernel, blocked QR or LU with narrow panels and
    the 16-column Cholesky panels."""
    A = gen_matrix(m, n, kappa, 211103 + n)
    Qd, Rd, info = tsqr.rxr_cholqr(dev(A), s, 11103, variant=variant, extra_pass=False)
    Q, R = host(Qd), host(Rd)
    assert int(info.item()) == 0
    ref = oracle.rxr_cholqr(A, s, 11103, variant=variant, extra_pass=False)
    ortho, res = oracle.orthogonality(Q), oracle.residual(A, Q, R)
    rd = rel_fro(R, ref["R"])
    print(f"m={m} n={n} s={s} kappa={kappa:g}: ortho={ortho:.2e} (oracle "
          f"{oracle.orthogonality(ref['Q']):.2e}) res={res:.2e} relR={rd:.2e}")
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    # one CholeskyQR pass on the preconditioned matrix: orthogonality ~ u cond(A1)^2, with
    # cond(A1) = O(1) for the Householder factor (Section 3); the LU factor's cond(A1) also
    # carries cond(L) of the sketch's L, so its single pass is held to the oracle's own
    # orthogonality instead; residual at the FP64 level either way
    ortho_o = oracle.orthogonality(ref["Q"])
    assert ortho <= (1e-12 if variant == tsqr.RQR else max(1e-12, 10 * ortho_o))
    assert res <= 1e-13
    assert rd <= 100 * n * EPS * kappa + 1e-14


def test_end_to_end_wide_full_size():
    """The wide configuration at full size (2^18 x 1024, s = 2048, kappa = 1e12, no extra
    pass): FP64 targets on the device metrics."""
    m, n, s = 1 << 18, 1024, 2048
    A = gen_matrix(m, n, 1e12, 211103)
    Ad = dev(A)
    del A
    Qd, Rd, info = tsqr.rxr_cholqr(Ad, s, 11103, extra_pass=False)
    assert int(info.item()) == 0
    ortho, res = gpu_orthogonality(Qd), gpu_residual(Ad, Qd, Rd)
    print(f"wide full size: ortho={ortho:.2e} res={res:.2e}")
    assert ortho <= 1e-12 and res <= 1e-13
    R = host(Rd)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)


@pytest.fixture(scope="module")
def tall128():
    m, n, s = 1 << 20, 128, 256
    A = gen_matrix(m, n, 1e14, 211102)
    return A, dev(A), s


@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
def test_end_to_end_tall128_full_size(tall128, variant):
    """The benchmark's workload (2^20 x 128, s = 256, kappa = 1e14, one extra pass) through
    the same explicit-workspace call the benchmark times: FP64 targets on the device
    metrics, R upper with a positive diagonal."""
    A, Ad, s = tall128
    m, n = A.shape
    work = tsqr.alloc_workspace(m, n, s)
    Qd, Rd, info = tsqr.rxr_cholqr(Ad, s, 11102, variant=variant, workspace=work)
    assert int(info.item()) == 0
    ortho, res = gpu_orthogonality(Qd), gpu_residual(Ad, Qd, Rd)
    print(f"tall128 variant={variant}: ortho={ortho:.2e} res={res:.2e}")
    assert ortho <= 1e-12 and res <= 1e-13
    R = host(Rd)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)


def test_tall128_sketch_sampled_rows(tall128):
    """Rows of the full-size sketch against the oracle's normals, one row at a time, and
    against the device's own normals at the FP64 summation bound."""
    A, Ad, s = tall128
    m = A.shape[0]
    Bg = host(tsqr.sketch(Ad, s, 11102))
    absA = np.abs(A)
    rs = 1.0 / math.sqrt(s)
    for i in (0, 63, 200, 255):
        z = oracle.sketch_normals(11102, i, 1, 0, m)[0]
        exact = rs * (z @ A)
        tol = rs * (NORMAL_ABS_TOL * absA.sum(axis=0) + 4 * m * U * (np.abs(z) @ absA))
        assert np.all(np.abs(Bg[i] - exact) <= tol), i
        # FP64 arithmetic of the product, against the normals the device generates
        zd = host(tsqr.sketch_normals(11102, i, 1, 0, m))
        ref = rs * (zd @ A)
        tol64 = fp64_sketch_tol(zd, A, s, ref)
        print(f"row {i}: max |B - rs z_dev A| / fp64 bound = {(np.abs(Bg[i] - ref[0]) / tol64[0]).max():.3e}")
        assert np.all(np.abs(Bg[i] - ref[0]) <= tol64[0]), i


def test_end_to_end_plain_forms_and_rless():
    m, n, s = 4096, 32, 64
    A = gen_matrix(m, n, 1e10, 211101)
    Ad = dev(A)
    for fn in (tsqr.rqr_cholqr, tsqr.rlu_cholqr):
        Qd, Rd = fn(Ad, s, 11101)
        _check_qr(A, Qd, Rd, host(Qd), host(Rd), 0)
    # R-less: Q identical to the full call
    Qa, Ra, _ = tsqr.rxr_cholqr(Ad, s, 11101)
    Qb, Rb, _ = tsqr.rxr_cholqr(Ad, s, 11101, want_r=False)
    assert Rb is None and torch.equal(Qa, Qb)


def test_end_to_end_no_extra_pass_and_ld():
    m, n, s = 5000, 48, 96
    A = gen_matrix(m, n, 1e9, 3)
    Qd, Rd, info = tsqr.rxr_cholqr(dev(A, ld=m + 11), s, 5, extra_pass=False)
    Q, R = host(Qd), host(Rd)
    assert int(info.item()) == 0
    ref = oracle.rxr_cholqr(A, s, 5, extra_pass=False)
    # one CholeskyQR pass on the preconditioned matrix: orthogonality ~ u cond(A1)^2
    assert oracle.orthogonality(Q) <= 1e-13
    assert oracle.residual(A, Q, R) <= 1e-13
    assert rel_fro(R, ref["R"]) <= 100 * n * EPS * 1e9


def test_end_to_end_deterministic():
    A = gen_matrix(20000, 64, 1e12, 8)
    Ad = dev(A)
    Q1, R1, _ = tsqr.rxr_cholqr(Ad, 128, 9)
    Q2, R2, _ = tsqr.rxr_cholqr(Ad, 128, 9)
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)


def test_end_to_end_breakdown_poisons():
    A = gen_matrix(2048, 16, 1e3, 4)
    A[:, 7] = 0.0
    Qd, Rd, info = tsqr.rxr_cholqr(dev(A), 32, 1)
    assert int(info.item()) == 1008
    assert torch.isnan(Qd).all() and torch.isnan(Rd).all()
    A2 = gen_matrix(2048, 16, 1e3, 4)
    A2[100, 3] = np.nan
    Qd2, Rd2, info2 = tsqr.rxr_cholqr(dev(A2), 32, 1)
    assert int(info2.item()) != 0
    assert torch.isnan(Qd2).all() and torch.isnan(Rd2).all()


def test_gpu_metrics_helper_matches_oracle():
    """The blocked FP64 metric of gpu_helpers agrees with the oracle's double-double one
    within its own rounding: a diagonal entry of a 4096-row block Gram carries about
    sqrt(4096) u, so the Frobenius norm over n diagonal entries about 2 sqrt(n) 64 u."""
    n = 40
    A = gen_matrix(9000, n, 1e8, 2)
    Qd, Rd, _ = tsqr.rxr_cholqr(dev(A), 2 * n, 2)
    Q, R = host(Qd), host(Rd)
    o1, o2 = gpu_orthogonality(Qd), oracle.orthogonality(Q)
    r1, r2 = gpu_residual(dev(A), Qd, Rd), oracle.residual(A, Q, R)
    assert abs(o1 - o2) <= 2 * math.sqrt(n) * 64 * U
    assert abs(r1 - r2) <= 0.05 * r2 + 64 * U
