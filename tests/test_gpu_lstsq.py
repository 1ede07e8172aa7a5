"""GPU parity of the least-squares solver preconditioned by the sketch's R factor (paper
Section 5.2), through the C ABI, against the CPU oracle's solver and the exact solution.

Both sides run the same algorithm; their x differ by rounding, amplified by cond(R0), so
the bar is ||x - x_oracle|| / ||x_oracle|| <= 100 kappa u, the forward-error level of the
method (pinned on the CPU against LAPACK).  A consistent system is also checked against
its exact solution at the same level.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2111_11148_amd as tsqr
from inputs import gen_matrix

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def _gpu(gpu_available):
    tsqr.load()
    torch.cuda.synchronize()
    yield


@pytest.mark.parametrize("sketch", ["gaussian", "rows"])
@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
@pytest.mark.parametrize("m,n,s,kappa", [(4096, 32, 64, 1e3), (4096, 32, 64, 1e10),
                                         (1027, 17, 40, 1e6), (6000, 128, 256, 1e8),
                                         (300, 1, 2, 1.0), (2000, 300, 600, 1e4)])
def test_lstsq_matches_oracle(sketch, variant, m, n, s, kappa):
    A = gen_matrix(m, n, kappa, 2111090 + m + n)
    rng = np.random.default_rng(m + n)
    xt = rng.standard_normal(n)
    b = A @ xt + 1e-3 * rng.standard_normal(m)
    xo, io = oracle.lstsq(A, b, s, 7, variant=variant, sketch=sketch)
    assert io == 0
    xd, info = tsqr.lstsq(tsqr.to_device_colmajor(A, ld=m + 2),
                          torch.from_numpy(b).cuda(), s, 7, variant=variant, sketch=sketch)
    assert int(info.item()) == 0
    x = xd.cpu().numpy()
    d = np.linalg.norm(x - xo) / np.linalg.norm(xo)
    print(f"lstsq {sketch} variant={variant} m={m} n={n} kappa={kappa:g}: rel diff {d:.2e}")
    assert d <= 100 * kappa * U


def test_lstsq_breakdown_gives_nan():
    A = gen_matrix(2048, 16, 1e3, 4)
    A[:, 7] = 0.0
    b = np.ones(2048)
    xd, info = tsqr.lstsq(tsqr.to_device_colmajor(A), torch.from_numpy(b).cuda(), 32, 1)
    _, io = oracle.lstsq(A, b, 32, 1)
    assert io // 1000 == 1 and int(info.item()) // 1000 == 1
    assert torch.isnan(xd).all()


def test_lstsq_full_size_consistent():
    """2^20 x 128 at kappa 1e10 with b = A x_true: x within 100 kappa u of x_true, with
    both sketches."""
    m, n = 1 << 20, 128
    A = gen_matrix(m, n, 1e10, 211109)
    xt = np.random.default_rng(3).standard_normal(n)
    b = torch.from_numpy(A @ xt).cuda()
    Ad = tsqr.to_device_colmajor(A)
    del A
    for sketch in ("gaussian", "rows"):
        xd, info = tsqr.lstsq(Ad, b, 256, 11, sketch=sketch)
        assert int(info.item()) == 0
        e = np.linalg.norm(xd.cpu().numpy() - xt) / np.linalg.norm(xt)
        print(f"lstsq full size {sketch}: forward error {e:.2e}")
        assert e <= 100 * 1e10 * U
