"""Device accuracy metrics (double-double ||Q^T Q - I||_F and ||A - QR||_F / ||A||_F, the
measures of paper Section 4.2) against closed forms and against the oracle's
double-double metrics (those are pinned against mpmath on the CPU)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2111_11148_amd as tsqr
from inputs.matrices import gen_matrix

pytestmark = pytest.mark.gpu


def test_metrics_closed_forms():
    # Q = (1 + d) [I; 0]: Q^T Q - I = (2d + d^2) I exactly (d = 2^-30), so the orthogonality
    # is sqrt(n) (2^-29 + 2^-60); A = Q with R = I leaves a residual of exactly 0.
    m, n = 3000, 37
    d = 2.0 ** -30
    Qh = np.zeros((m, n), order="F")
    Qh[np.arange(n), np.arange(n)] = 1.0 + d
    Q = tsqr.to_device_colmajor(Qh)
    R = tsqr.to_device_colmajor(np.eye(n))
    o, r = tsqr.metrics(Q, Q, R)
    assert o == pytest.approx(np.sqrt(n) * (2.0 ** -29 + 2.0 ** -60), rel=1e-14)
    assert r == 0.0
    # the residual of an exact integer product is 0; one entry off by 1 gives 1/||A||_F
    rng = np.random.default_rng(3)
    Qi = rng.integers(-8, 9, size=(m, n)).astype(np.float64)
    Ri = np.triu(rng.integers(-8, 9, size=(n, n)).astype(np.float64))
    Ai = Qi @ Ri  # exact: every partial sum is a small integer
    o2, r2 = tsqr.metrics(tsqr.to_device_colmajor(Qi), tsqr.to_device_colmajor(Ai),
                          tsqr.to_device_colmajor(Ri))
    assert r2 == 0.0
    Ai[17, 5] += 1.0
    _, r3 = tsqr.metrics(tsqr.to_device_colmajor(Qi), tsqr.to_device_colmajor(Ai),
                         tsqr.to_device_colmajor(Ri))
    assert r3 == pytest.approx(1.0 / np.linalg.norm(Ai), rel=1e-14)
    # orthogonality of the integer Q: ||Q^T Q - I||_F exactly from integer arithmetic
    G = Qi.T @ Qi - np.eye(n)
    assert o2 == pytest.approx(np.sqrt(np.sum(G * G)), rel=1e-14)
    # no A: the residual is not computed
    o4, r4 = tsqr.metrics(Q)
    assert o4 == o and np.isnan(r4)


@pytest.mark.parametrize("m,n,kappa", [(4096, 32, 1e10), (5000, 100, 1e6), (70001, 128, 1e14),
                                       (1000, 1, 1.0), (3333, 17, 1e3)])
def test_metrics_match_oracle(m, n, kappa):
    A_h = gen_matrix(m, n, kappa, 77 + n)
    A = tsqr.to_device_colmajor(A_h)
    Q, R, info = tsqr.rxr_cholqr(A, 2 * n, 5, extra_pass=True)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Qh = np.asfortranarray(Q.cpu().numpy())
    Rh = np.asfortranarray(R.cpu().numpy())
    o, r = tsqr.metrics(Q, A, R)
    o_ref, r_ref = oracle.orthogonality(Qh), oracle.residual(A_h, Qh, Rh)
    print(f"m={m} n={n} kappa={kappa:g}: ortho {o:.6e} (oracle {o_ref:.6e}), "
          f"residual {r:.6e} (oracle {r_ref:.6e})")
    # both are accurate to about m u^2 relative to the sum of |terms|
    assert o == pytest.approx(o_ref, rel=1e-9)
    assert r == pytest.approx(r_ref, rel=1e-9)
    # repeatable bit for bit
    assert tsqr.metrics(Q, A, R) == (o, r)
