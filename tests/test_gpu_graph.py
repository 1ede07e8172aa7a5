"""The single-problem chain captured into a HIP graph: every replay gives the eager call's
Q, R and info bit for bit, with eager work and synchronizations between the replays (the
chain records kernels and copies only; its counters are cleared by a kernel)."""
import numpy as np
import pytest
import torch

import paper_2111_11148_amd as tsqr
from inputs.matrices import gen_matrix

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant,sketch,n", [(tsqr.RQR, "gaussian", 64), (tsqr.RLU, "gaussian", 100),
                                              (tsqr.RQR, "rows", 128)])
def test_chain_graph_replays_match_eager(variant, sketch, n):
    m, s, seed = 30000, 2 * n, 31 + n
    A = tsqr.to_device_colmajor(gen_matrix(m, n, 1e10, 301 + n))
    work = tsqr.alloc_workspace(m, n, s)
    Qe, Re, ie = tsqr.rxr_cholqr(A, s, seed, variant=variant, workspace=work, sketch=sketch)
    torch.cuda.synchronize()
    assert int(ie.item()) == 0
    Q, R = tsqr.colmajor(m, n), tsqr.colmajor(n, n)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):  # warm-up outside the capture
        tsqr.rxr_cholqr(A, s, seed, variant=variant, Q=Q, R=R, workspace=work, info=info,
                        stream=st, sketch=sketch)
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        tsqr.rxr_cholqr(A, s, seed, variant=variant, Q=Q, R=R, workspace=work, info=info,
                        stream=st, sketch=sketch)
    other = tsqr.alloc_workspace(m, n, s)
    for rep in range(3):
        Q.fill_(np.nan)
        R.fill_(np.nan)
        info.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(info.item()) == 0, rep
        assert torch.equal(Q, Qe) and torch.equal(R, Re), rep
        # eager work between the replays, on its own workspace
        tsqr.rxr_cholqr(A, s, seed + 1, variant=variant, workspace=other, sketch=sketch)
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec,kappa", [(tsqr.FP32, 1e4), (tsqr.FP32, 1e10), (tsqr.BF16, 1e8),
                                        (tsqr.BF16, 1e13)])
def test_mixed_automatic_chain_graph_replays_match_eager(prec, kappa):
    """The automatic mixed-precision chain decides its stage and its passes on the device,
    so it can be captured: every replay reproduces the eager Q, R, info and report (passes,
    stage) bit for bit, whatever number of passes the input needs."""
    m, n, s, seed = 30000, 64, 128, 17
    A = tsqr.to_device_colmajor(gen_matrix(m, n, kappa, 401))
    ws = torch.empty(tsqr.mixed_workspace_bytes(m, n, s, prec), dtype=torch.uint8, device="cuda")
    Qe, Re, ie, re = tsqr.rxr_cholqr_mixed(A, s, seed, prec, workspace=ws)
    torch.cuda.synchronize()
    assert int(ie.item()) == 0
    print(f"prec={prec} kappa={kappa:g}: passes={int(re[0])} stage={int(re[1])}")
    Q, R = tsqr.colmajor(m, n), tsqr.colmajor(n, n)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    rep_t = torch.zeros(2, dtype=torch.int32, device="cuda")
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        tsqr.rxr_cholqr_mixed(A, s, seed, prec, Q=Q, R=R, workspace=ws, info=info, report=rep_t,
                              stream=st)
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        tsqr.rxr_cholqr_mixed(A, s, seed, prec, Q=Q, R=R, workspace=ws, info=info, report=rep_t,
                              stream=st)
    other = torch.empty_like(ws)
    for r in range(3):
        Q.fill_(np.nan)
        R.fill_(np.nan)
        info.fill_(-7)
        rep_t.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(info.item()) == 0, r
        assert torch.equal(rep_t, re), r
        assert torch.equal(Q, Qe) and torch.equal(R, Re), r
        # eager work between the replays (another seed, its own workspace)
        tsqr.rxr_cholqr_mixed(A, s, seed + 1, prec, workspace=other)
        torch.cuda.synchronize()
