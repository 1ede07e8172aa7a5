"""GPU parity of the mixed-precision variant (FP32 / BF16 inputs on the matrix cores,
FP64 CholeskyQR passes) against the CPU oracle, through the C ABI.

Step tests compare each low-precision kernel with the oracle's exact (FP64-summed) sum of
the same rounded inputs; the device adds FP32 accumulation error, bounded per entry by
GAMMA32 * sum |terms| (FP32 sums over at most 64 terms before each FP64 flush), and, in
the sketch, the device's FP32 normals may differ from the oracle's by NORMAL_ABS_TOL before
rounding (for BF16 that can move a normal by one BF16 step; the bound takes the largest
such move that is possible for each normal).  End-to-end tests check the FP64-accurate
results the mixed variant is for: orthogonality and residual at the FP64 targets, R within
the perturbation bound of the oracle's FP64 R, and the same number of FP64 passes.
"""
import math

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
U32 = 2.0 ** -24
# FP32 accumulation: at most 64 rounded additions (each MFMA step rounds once) per FP64
# flush, plus the rounding of the products for the FP32 inputs; 70 covers both.
GAMMA32 = 70 * U32
NORMAL_ABS_TOL = 2e-5  # device FP32 normal vs oracle FP64 normal (see test_gpu_parity)
PRECS = [tsqr.FP32, tsqr.BF16]


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    tsqr.load()
    torch.cuda.synchronize()
    yield


def dev(A, ld=None):
    return tsqr.to_device_colmajor(A, ld=ld)


def rnd(x, prec):
    """Round to FP32, then (BF16) to BF16, both to nearest even (torch's conversions)."""
    t = torch.as_tensor(np.asarray(x, dtype=np.float64)).to(torch.float32)
    if prec == tsqr.BF16:
        t = t.to(torch.bfloat16).to(torch.float32)
    return t.to(torch.float64).numpy()


def normal_uncertainty(Zo, prec):
    """Largest |r(z_dev) - r(r32(z_oracle))| possible when |z_dev - z_oracle| <= tol."""
    d = NORMAL_ABS_TOL + 2 * U32 * np.abs(Zo)
    ref = rnd(Zo, prec)
    return np.maximum(np.abs(rnd(Zo + d, prec) - ref), np.abs(rnd(Zo - d, prec) - ref)) + \
        (d if prec == tsqr.FP32 else 0.0)


def worst(err, tol, got, exp, mag, k=4):
    """Print the entries that exceed their bound most (index, device, oracle, sum |terms|)."""
    r = (err / tol).ravel(order="F")
    for f in np.argsort(r)[::-1][:k]:
        i, j = np.unravel_index(f, err.shape, order="F")
        print(f"  ({i},{j}) ratio {r[f]:.3g} dev {got[i, j]:.9g} oracle {exp[i, j]:.9g} "
              f"sum|terms| {mag[i, j]:.4g}")


def to_lowp_device(Xh, prec):
    """Column-major device tensor of the (exactly representable) values Xh."""
    m, n = Xh.shape
    dt = torch.float32 if prec == tsqr.FP32 else torch.bfloat16
    X = tsqr.colmajor(m, n, device="cuda", dtype=dt)
    X.copy_(torch.from_numpy(np.ascontiguousarray(Xh)).to(torch.float32).to(dt))
    return X


# ---------------------------------------------------------------------------- sketch --
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("m,n,s", [(4096, 32, 64), (1000, 5, 7), (1027, 17, 40), (3000, 128, 256),
                                   (777, 1, 1), (2050, 100, 100), (4100, 256, 512),
                                   (3001, 200, 300), (5000, 144, 150), (700, 130, 20)])
def test_sketch_lowp_parity(prec, m, n, s):
    A = gen_matrix(m, n, 1e6, 400 + m)
    seed = 11104 + n
    Bg = host(tsqr.sketch_lowp(dev(A), s, seed, prec))
    Bo = oracle.sketch_apply_lowp(prec, A, s, seed)
    Zo = oracle.sketch_normals(seed, 0, s, 0, m)
    Ap = np.abs(rnd(A, tsqr.FP32))  # A enters the sketch as FP32 for both input types
    Zp = np.abs(rnd(Zo, prec))
    Dz = normal_uncertainty(Zo, prec)
    rs = 1.0 / math.sqrt(s)
    tol = rs * (Dz @ Ap + GAMMA32 * ((Zp + Dz) @ Ap)) + 4 * m * U * np.abs(Bo)
    err = np.abs(Bg - Bo)
    print(f"prec={prec} m={m} n={n} s={s}: max err {err.max():.3e}, max err/tol "
          f"{(err / tol).max():.3f}")
    assert np.all(err <= tol)
    # against the normals the device generates: only the device's FP32 product rounding
    # and accumulation remain (GAMMA32); products of two FP32 numbers are exact in FP64,
    # so the reference below is exact up to its own FP64 sum (4 m u)
    Zd = rnd(host(tsqr.sketch_normals(seed, 0, s, 0, m)), prec)
    ref = rs * (Zd @ rnd(A, tsqr.FP32))
    tol_d = rs * GAMMA32 * (np.abs(Zd) @ Ap) + 4 * m * U * np.abs(ref)
    err_d = np.abs(Bg - ref)
    print(f"  against device normals: max err/tol {(err_d / tol_d).max():.3f}")
    assert np.all(err_d <= tol_d)


def test_sketch_lowp_leading_dimension_and_determinism():
    m, n, s = 2000, 24, 48
    A = gen_matrix(m, n, 1e3, 5)
    for prec in PRECS:
        B1 = host(tsqr.sketch_lowp(dev(A), s, 3, prec))
        B2 = host(tsqr.sketch_lowp(dev(A, ld=m + 37), s, 3, prec))
        assert np.array_equal(B1, B2)


# ----------------------------------------------------------------------------- apply --
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("m,n", [(4096, 32), (1000, 5), (1027, 17), (5000, 128), (333, 1),
                                 (2049, 100), (3001, 256), (100, 16), (200, 48)])
def test_apply_rinv_lowp_parity(prec, m, n):
    """X = r(r(Y) r(Rinv)): the device's FP32 sum differs from the exact one by at most
    GAMMA32 sum_k |Y_ik Rinv_kc|; both are then rounded to the output type, which may
    differ by one rounding step of the type on either side (2 u_p |X|)."""
    A = gen_matrix(m, n, 1e6, 500 + m)
    s = 2 * n
    B = oracle.sketch_apply(A, s, 9)
    R0, info = oracle.householder_r(B)
    assert info == 0
    Rinv = oracle.trtri_upper(R0)
    Xg = tsqr.apply_rinv_lowp(dev(A), dev(Rinv), prec)
    assert Xg.dtype == (torch.float32 if prec == tsqr.FP32 else torch.bfloat16)
    Xg = host(Xg.to(torch.float64))
    Xo = oracle.apply_rinv_lowp(prec, A, Rinv)
    up = U32 if prec == tsqr.FP32 else 2.0 ** -8
    mag = np.abs(rnd(A, prec)) @ np.abs(rnd(np.triu(Rinv), prec))
    tol = (1 + up) * GAMMA32 * mag + 2 * up * np.abs(Xo) + 1e-300
    err = np.abs(Xg - Xo)
    print(f"prec={prec} m={m} n={n}: max err/tol {(err / tol).max():.3f}")
    worst(err, tol, Xg, Xo, mag)
    bad = err > tol
    if bad.any():
        rows, cols = np.nonzero(bad)
        print(f"  {bad.sum()} bad entries; rows {np.unique(rows % 16)} (mod 16), "
              f"cols {np.unique(cols)}")
    assert np.all(err <= tol)


# ------------------------------------------------------------------------------ gram --
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("m,n", [(4096, 32), (1000, 5), (1027, 17), (6000, 128), (129, 1),
                                 (20000, 64), (3001, 256), (65, 200)])
def test_gram_lowp_parity(prec, m, n):
    """W = X^T X of a low-precision X: |W_dev - W_exact| <= GAMMA32 |X|^T |X| (+ FP64)."""
    rng = np.random.default_rng(m + n)
    Xh = rnd(rng.standard_normal((m, n)) * (1 + np.arange(n))[None, :], prec)
    Wg = host(tsqr.gram_lowp(to_lowp_device(Xh, prec), prec))
    Wo = oracle.gram_lowp(prec, np.asfortranarray(Xh))
    mag = np.abs(Xh).T @ np.abs(Xh)
    tol = GAMMA32 * mag + 4 * m * U * mag
    assert np.array_equal(Wg, Wg.T)
    err = np.abs(Wg - Wo)
    print(f"prec={prec} m={m} n={n}: max err/tol {(err / tol).max():.3f}")
    assert np.all(err <= tol)


# ------------------------------------------------------------------------ end to end --
def _qr_checks(A, Qd, Rd, info, ortho_tol=1e-12, res_tol=1e-13):
    assert int(info.item()) == 0
    Q, R = host(Qd), host(Rd)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    ortho, res = oracle.orthogonality(Q), oracle.residual(A, Q, R)
    assert ortho <= ortho_tol, ortho
    assert res <= res_tol, res
    return Q, R, ortho, res


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
@pytest.mark.parametrize("m,n,s,kappa", [(4096, 32, 64, 1e4), (4096, 32, 64, 1e8),
                                         (4096, 32, 64, 1e12), (1027, 17, 40, 1e10),
                                         (6000, 128, 256, 1e12), (8192, 256, 512, 1e8),
                                         (300, 1, 2, 1.0), (2500, 100, 200, 1e6)])
def test_mixed_end_to_end_auto(prec, variant, m, n, s, kappa):
    """Automatic FP64 passes: FP64 targets met, R within c kappa u of the FP64 oracle's R,
    and the same number of FP64 passes as the oracle's mixed method."""
    A = gen_matrix(m, n, kappa, 2111040 + m + n)
    seed = 11104 + n
    Qd, Rd, info, rep = tsqr.rxr_cholqr_mixed(dev(A), s, seed, prec, variant=variant,
                                              fp64_passes=0)
    passes, stage = (int(v) for v in rep.cpu())
    Q, R, ortho, res = _qr_checks(A, Qd, Rd, info)
    ref64 = oracle.rxr_cholqr(A, s, seed, variant=variant)
    refmx = oracle.rxr_cholqr_mixed(A, s, seed, prec=prec, variant=variant, fp64_passes=0)
    assert ref64["info"] == 0 and refmx["info"] == 0
    rd = rel_fro(R, ref64["R"])
    print(f"prec={prec} variant={variant} m={m} n={n} kappa={kappa:g}: passes={passes} "
          f"(oracle {refmx['passes']}) ortho={ortho:.2e} res={res:.2e} relR={rd:.2e}")
    assert passes == refmx["passes"]
    assert stage == (1 if refmx["lp_info"] >= 0 else 0)
    assert rd <= 100 * n * EPS * kappa + 1e-14


@pytest.mark.parametrize("prec,passes,kappa", [(tsqr.FP32, 1, 1e4), (tsqr.FP32, 1, 1e6),
                                               (tsqr.FP32, 2, 1e10), (tsqr.BF16, 2, 1e4),
                                               (tsqr.BF16, 3, 1e8)])
def test_mixed_end_to_end_fixed_passes(prec, passes, kappa):
    m, n, s = 5000, 48, 96
    A = gen_matrix(m, n, kappa, 77)
    ref = oracle.rxr_cholqr_mixed(A, s, 5, prec=prec, fp64_passes=passes)
    assert ref["info"] == 0 and ref["passes"] == passes
    assert oracle.orthogonality(ref["Q"]) <= 1e-12
    Qd, Rd, info, got = tsqr.rxr_cholqr_mixed(dev(A, ld=m + 3), s, 5, prec, fp64_passes=passes)
    assert int(got[0].item()) == passes and int(got[1].item()) == 1
    Q, R, _, _ = _qr_checks(A, Qd, Rd, info)
    assert rel_fro(R, ref["R"]) <= 100 * n * EPS * kappa + 1e-14


def test_mixed_low_precision_breakdown_falls_back():
    """Two columns an FP32 number apart by a factor 1 + 2^-30 (distinct in FP64, equal in
    FP32, the stage's input type); whether or not the stage's Cholesky breaks down on the
    device, the FP64 passes deliver an orthonormal Q (the oracle's mixed method breaks down
    there with the BF16 sketch's R0 and falls back to R0).  Three fixed passes, which
    always run the low-precision stage; the automatic mode skips it for this input."""
    A = gen_matrix(4096, 32, 1e3, 5)
    A[:, 4] = rnd(A[:, 4], tsqr.FP32)
    A[:, 5] = A[:, 4] * (1 + 2.0 ** -30)
    ref = oracle.rxr_cholqr_mixed(A, 64, 7, prec=tsqr.BF16, fp64_passes=3)
    assert ref["info"] == 0 and ref["lp_info"] > 0
    for prec in PRECS:
        print(f"prec={prec}", flush=True)
        Qd, Rd, info, passes = tsqr.rxr_cholqr_mixed(dev(A), 64, 7, prec, fp64_passes=3)
        assert int(info.item()) == 0 and int(passes[0].item()) == 3
        assert oracle.orthogonality(host(Qd)) <= 1e-13
        # automatic mode: the stage is skipped (oracle lp_info -1); this nearly singular
        # input sits at the edge of the pass rule, so only the outcome is compared, not the
        # count
        Qa, Ra, infoa, pa = tsqr.rxr_cholqr_mixed(dev(A), 64, 7, prec, fp64_passes=0)
        refa = oracle.rxr_cholqr_mixed(A, 64, 7, prec=prec, fp64_passes=0)
        assert refa["lp_info"] == -1 and int(infoa.item()) == 0 and 1 <= int(pa[0].item()) <= 3
        assert int(pa[1].item()) == 0
        assert oracle.orthogonality(host(Qa)) <= 1e-13


def test_mixed_deterministic_and_rless():
    A = gen_matrix(20000, 64, 1e10, 8)
    Ad = dev(A)
    for prec in PRECS:
        Q1, R1, _, p1 = tsqr.rxr_cholqr_mixed(Ad, 128, 9, prec)
        Q2, R2, _, p2 = tsqr.rxr_cholqr_mixed(Ad, 128, 9, prec)
        assert torch.equal(p1, p2) and torch.equal(Q1, Q2) and torch.equal(R1, R2)
        Q3, R3, _, _ = tsqr.rxr_cholqr_mixed(Ad, 128, 9, prec, want_r=False)
        assert R3 is None and torch.equal(Q1, Q3)


def test_mixed_breakdown_poisons():
    A = gen_matrix(2048, 16, 1e3, 4)
    A[:, 7] = 0.0
    for prec in PRECS:
        Qd, Rd, info, _ = tsqr.rxr_cholqr_mixed(dev(A), 32, 1, prec)
        assert int(info.item()) == 1008
        assert torch.isnan(Qd).all() and torch.isnan(Rd).all()


def test_mixed_workspace_too_small_is_an_error():
    A = dev(gen_matrix(1000, 8, 10.0, 1))
    nbytes = tsqr.mixed_workspace_bytes(1000, 8, 16, tsqr.FP32)
    ws = torch.empty(nbytes - 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(tsqr.TsqrError):
        tsqr.rxr_cholqr_mixed(A, 16, 1, tsqr.FP32, workspace=ws)


# -------------------------------------------------- full size: 2^20 x 256, sketch 512 --
@pytest.fixture(scope="module")
def big_mixed():
    m, n, s = 1 << 20, 256, 512
    A = gen_matrix(m, n, 1e8, 2111041)
    return A, dev(A), s


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_full_size_properties(big_mixed, prec):
    """The workload the benchmark times: FP64 targets on the device metrics."""
    A, Ad, s = big_mixed
    Qd, Rd, info, passes = tsqr.rxr_cholqr_mixed(Ad, s, 11104, prec)
    assert int(info.item()) == 0
    ortho, res = gpu_orthogonality(Qd), gpu_residual(Ad, Qd, Rd)
    print(f"prec={prec}: passes={passes} ortho={ortho:.2e} res={res:.2e}")
    assert ortho <= 1e-12 and res <= 1e-13
    R = host(Rd)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)


@pytest.mark.parametrize("prec", PRECS)
def test_mixed_full_size_sketch_sampled_rows(big_mixed, prec):
    """Rows of the low-precision sketch at full size against the oracle's definition,
    computed one row at a time from the oracle's normals."""
    A, Ad, s = big_mixed
    seed = 11104
    Bg = host(tsqr.sketch_lowp(Ad, s, seed, prec))
    Ap = rnd(A, tsqr.FP32)  # A enters the sketch as FP32 for both input types
    absAp = np.abs(Ap)
    rs = 1.0 / math.sqrt(s)
    m = A.shape[0]
    for i in (0, 17, 255, 511):
        z = oracle.sketch_normals(seed, i, 1, 0, m)[0]
        zr = rnd(z, prec)
        exact = rs * (zr @ Ap)
        dz = normal_uncertainty(z, prec)
        tol = rs * (dz @ absAp + GAMMA32 * ((np.abs(zr) + dz) @ absAp)) + \
            4 * m * U * rs * (np.abs(zr) @ absAp)
        assert np.all(np.abs(Bg[i] - exact) <= tol), i
