"""Calls on a side stream with no caller workspace: the binding allocates its outputs and
temporaries on that stream, so allocations made on the current stream right after the
call cannot reuse memory the side stream's kernels still use.  The results equal those of
the same call on the current stream, bit for bit."""
import numpy as np
import pytest
import torch

import paper_2111_11148_amd as tsqr
from inputs.matrices import gen_matrix

pytestmark = pytest.mark.gpu


def _scribble():
    # allocations on the current stream, written at once
    return [torch.full((1 << 21,), float("nan"), dtype=torch.float64, device="cuda")
            for _ in range(16)]


def test_side_stream_calls_without_workspace():
    m, n, s, seed = 60000, 64, 128, 5
    A = tsqr.to_device_colmajor(gen_matrix(m, n, 1e10, 77))
    Qr, Rr, ir = tsqr.rxr_cholqr(A, s, seed)
    Br = tsqr.sketch(A, s, seed)
    Xr = tsqr.trsm(A, Rr)
    Wr = tsqr.gram(Qr)
    Qm, Rm, im, pm = tsqr.rxr_cholqr_mixed(A, s, seed, lowp=tsqr.FP32, fp64_passes=2)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    for rep in range(2):
        side.wait_stream(torch.cuda.current_stream())
        Q, R, info = tsqr.rxr_cholqr(A, s, seed, stream=side)
        junk = _scribble()
        B = tsqr.sketch(A, s, seed, stream=side)
        junk += _scribble()
        X = tsqr.trsm(A, Rr, stream=side)
        junk += _scribble()
        W = tsqr.gram(Qr, stream=side)
        junk += _scribble()
        Q2, R2, i2, p2 = tsqr.rxr_cholqr_mixed(A, s, seed, lowp=tsqr.FP32, fp64_passes=2,
                                               stream=side)
        junk += _scribble()
        torch.cuda.synchronize()
        del junk
        assert int(info.item()) == int(ir.item()) == 0
        assert torch.equal(Q, Qr) and torch.equal(R, Rr), rep
        assert torch.equal(B, Br) and torch.equal(X, Xr) and torch.equal(W, Wr), rep
        assert torch.equal(Q2, Qm) and torch.equal(R2, Rm) and torch.equal(p2, pm), rep
