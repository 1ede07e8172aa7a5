"""The no-allocation entry point (tsqr_rxr_cholqr_noalloc) against the explicit-workspace
one on the same inputs: identical kernels on identical inputs, so Q, R and info agree bit
for bit; two calls in a row (the second smaller) show the shared scratch array keeps no
state that changes a result.  Sizes beyond the array are refused before any work is
enqueued (a host check, covered in test_abi.py)."""
import numpy as np
import pytest
import torch

import paper_2111_11148_amd as tsqr
from inputs.matrices import gen_matrix

pytestmark = pytest.mark.gpu


def _ws_call(A, s, seed, variant, extra_pass):
    m, n = A.shape
    Q, R = tsqr.colmajor(m, n), tsqr.colmajor(n, n)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    tsqr.rxr_cholqr(A, s, seed, variant=variant, extra_pass=extra_pass, Q=Q, R=R, info=info)
    return Q, R, info


def _noalloc_call(A, s, seed, variant, extra_pass, with_info=True):
    m, n = A.shape
    Q, R = tsqr.colmajor(m, n, fill=7.0), tsqr.colmajor(n, n, fill=7.0)
    info = torch.full((1,), 99, dtype=torch.int32, device="cuda") if with_info else None
    tsqr.rxr_cholqr_noalloc(A, s, seed, Q, R, info, variant=variant, extra_pass=extra_pass)
    return Q, R, info


@pytest.mark.parametrize("variant", [tsqr.RQR, tsqr.RLU])
def test_noalloc_matches_workspace_form_two_calls(variant):
    cases = [(1 << 20, 128, 256, 1e14, 211102, 11102), (5000, 40, 80, 1e8, 9, 77)]
    for m, n, s, kappa, gseed, seed in cases:
        print(f"noalloc variant={variant} m={m} n={n} s={s}", flush=True)
        A = tsqr.to_device_colmajor(gen_matrix(m, n, kappa, gseed))
        Qw, Rw, iw = _ws_call(A, s, seed, variant, True)
        Qn, Rn, inf = _noalloc_call(A, s, seed, variant, True)
        torch.cuda.synchronize()
        assert int(iw.item()) == 0 and int(inf.item()) == 0
        assert torch.equal(Qn, Qw) and torch.equal(Rn, Rw)
        del A, Qw, Rw, Qn, Rn


def test_noalloc_without_info_and_breakdown():
    # R-less call without an info word, then a breakdown (a zero column) after it: the
    # second call reports the same info as the workspace form and leaves NaN outputs
    m, n, s = 4096, 32, 64
    A_h = gen_matrix(m, n, 1e6, 5)
    A = tsqr.to_device_colmajor(A_h)
    Qw, _, _ = _ws_call(A, s, 3, tsqr.RQR, False)
    Qn = tsqr.colmajor(m, n)
    tsqr.rxr_cholqr_noalloc(A, s, 3, Qn, None, None, extra_pass=False)
    torch.cuda.synchronize()
    assert torch.equal(Qn, Qw)
    A_h[:, 7] = 0.0
    Az = tsqr.to_device_colmajor(A_h)
    _, _, iw = _ws_call(Az, s, 3, tsqr.RQR, True)
    Qz, Rz, iz = _noalloc_call(Az, s, 3, tsqr.RQR, True)
    torch.cuda.synchronize()
    assert int(iz.item()) == int(iw.item()) == 1008
    assert bool(torch.isnan(Qz).all()) and bool(torch.isnan(Rz).all())

