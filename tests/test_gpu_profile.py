"""Phase timing of the C ABI: every launch of a chain is recorded under its phase name, in
launch order, with a positive duration; a filter keeps only the named phase."""
import pytest
import torch

import paper_2111_11148_amd as tsqr
from inputs.matrices import gen_matrix

pytestmark = pytest.mark.gpu

CHAIN = ["sketch", "sketch_reduce", "sketch_qr", "trsm_prep_r0", "trsm_r0", "gram1",
         "gram1_reduce", "potrf1", "trsm_prep_r1", "trsm_r1", "gram2", "gram2_reduce", "potrf2",
         "trsm_prep_r2", "trsm_r2", "trmm", "trmm", "poison"]


def test_profile_records_and_filter():
    m, n, s = 20000, 64, 128
    A = tsqr.to_device_colmajor(gen_matrix(m, n, 1e6, 41))
    work = tsqr.alloc_workspace(m, n, s)
    Q, R = tsqr.colmajor(m, n), tsqr.colmajor(n, n)
    info = torch.zeros(1, dtype=torch.int32, device="cuda")

    def step():
        tsqr.rxr_cholqr(A, s, 5, Q=Q, R=R, workspace=work, info=info)

    step()
    torch.cuda.synchronize()
    tsqr.profile_start()
    step()
    step()
    recs = tsqr.profile_stop()
    names = [r[0] for r in recs]
    assert names == CHAIN + CHAIN
    assert all(ms > 0.0 for _, ms in recs)

    tsqr.profile_start(only="trsm_r1")
    step()
    step()
    recs = tsqr.profile_stop()
    assert [r[0] for r in recs] == ["trsm_r1", "trsm_r1"]

    step()  # recording is off: nothing is kept
    tsqr.profile_start()
    recs = tsqr.profile_stop()
    assert recs == []
