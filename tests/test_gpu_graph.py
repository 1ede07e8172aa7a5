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
