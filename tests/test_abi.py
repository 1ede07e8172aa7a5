"""The C ABI library loads, exports every function include/tsqr.h declares, and rejects
invalid arguments synchronously with the documented LAPACK-style codes (host logic only:
no kernel is launched by any call here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tsqr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tsqr_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2111_11148_amd as tsqr

    return tsqr.load()


def test_header_declares_the_method_entry_points():
    names = declared_functions()
    for required in ("tsqr_rqr_cholqr", "tsqr_rlu_cholqr", "tsqr_rxr_cholqr_ws",
                     "tsqr_workspace_bytes", "tsqr_sketch", "tsqr_sketch_factor", "tsqr_trsm",
                     "tsqr_gram", "tsqr_potrf", "tsqr_trmm_upper"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert b"gfx950" in lib.tsqr_version()


def test_plain_form_argument_codes(lib):
    f = lib.tsqr_rqr_cholqr
    A = ctypes.c_void_p(0x10000000)
    Q = ctypes.c_void_p(0x20000000)
    R = ctypes.c_void_p(0x30000000)
    assert f(0, 1, A, 1, 1, 0, Q, R, None) == -1          # m < 1
    assert f(4, 8, A, 4, 8, 0, Q, R, None) == -1          # m < n
    assert f(8, 0, A, 8, 1, 0, Q, R, None) == -2          # n < 1
    assert f(8, 4, None, 8, 8, 0, Q, R, None) == -3       # A NULL
    assert f(8, 4, A, 7, 8, 0, Q, R, None) == -4          # lda < m
    assert f(8, 4, A, 8, 3, 0, Q, R, None) == -5          # s < n (the paper needs l >= n)
    assert f(8, 4, A, 8, 9000, 0, Q, R, None) == -5       # s above the supported maximum
    assert f(8, 4, A, 8, 8, 0, None, R, None) == -7       # Q NULL
    assert f(8, 4, A, 8, 8, 0, ctypes.c_void_p(0x10000008), R, None) == -7  # Q overlaps A
    assert f(8, 4, A, 8, 8, 0, Q, ctypes.c_void_p(0x20000010), None) == -8  # R overlaps Q
    assert lib.tsqr_rlu_cholqr(8, 4, A, 7, 8, 0, Q, R, None) == -4


def test_workspace_form_argument_codes(lib):
    f = lib.tsqr_rxr_cholqr_ws
    A, Q, R, W = (ctypes.c_void_p(x) for x in (0x10000000, 0x20000000, 0x30000000, 0x40000000))
    ok = dict(variant=0, m=64, n=8, A=A, lda=64, s=16, seed=1, extra=1, Q=Q, ldq=64, R=R, ldr=8,
              work=W, wb=1, info=None, st=None)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["variant"], a["m"], a["n"], a["A"], a["lda"], a["s"], a["seed"], a["extra"],
                 a["Q"], a["ldq"], a["R"], a["ldr"], a["work"], a["wb"], a["info"], a["st"])

    assert call(variant=2) == -1
    assert call(m=0) == -2
    assert call(n=0) == -3
    assert call(A=None) == -4
    assert call(lda=10) == -5
    assert call(s=7) == -6
    assert call(Q=None) == -9
    assert call(ldq=10) == -10
    assert call(ldr=7) == -12
    assert call(work=None) == -13
    assert call() == -101  # TSQR_ERR_WORKSPACE: 1 byte is too small
    assert call(m=3000, lda=3000, ldq=3000, n=1100, s=2200, ldr=1100) == -102  # too wide


def test_workspace_bytes_monotone(lib):
    lib.tsqr_workspace_bytes.restype = ctypes.c_size_t
    assert lib.tsqr_workspace_bytes(100, 0, 1) == 0
    assert lib.tsqr_workspace_bytes(10, 20, 20) == 0
    small = lib.tsqr_workspace_bytes(4096, 32, 64)
    big = lib.tsqr_workspace_bytes(1 << 20, 128, 256)
    assert 0 < small < big


def test_batched_descriptor_validation(lib):
    """Host-only checks of the batched entry points: invalid problems give a zero workspace
    size and argument codes, before any device work."""
    import paper_2111_11148_amd as tsqr

    P = tsqr._Problem
    good = P(1000, 32, 1000, 64, 1, 16, 1 << 20, 1000, 0, 32)  # fake, non-null pointers
    arr = (P * 2)(good, good)
    assert lib.tsqr_batched_workspace_bytes(2, ctypes.cast(arr, ctypes.c_void_p)) > 0
    for bad in (P(1000, 129, 1000, 258, 1, 16, 32, 1000, 0, 129),   # n > 128
                P(1000, 32, 1000, 600, 1, 16, 32, 1000, 0, 32),     # s > 512
                P(1000, 32, 1000, 16, 1, 16, 32, 1000, 0, 32),      # s < n
                P(1000, 32, 999, 64, 1, 16, 32, 1000, 0, 32),       # lda < m
                P(1000, 32, 1000, 64, 1, 0, 32, 1000, 0, 32),       # A null
                P(20, 32, 20, 64, 1, 16, 32, 20, 0, 32),            # m < n
                P(1000, 100, 1000, 300, 1, 16, 32, 1000, 0, 100)):  # s > 256 with n > 64
        arr = (P * 2)(good, bad)
        assert lib.tsqr_batched_workspace_bytes(2, ctypes.cast(arr, ctypes.c_void_p)) == 0
        plan = ctypes.c_void_p()
        rc = lib.tsqr_batched_create(0, 0, 2, ctypes.cast(arr, ctypes.c_void_p), 16, 1 << 30,
                                     16, None, ctypes.byref(plan))
        assert rc == -4 and plan.value is None
    assert lib.tsqr_batched_workspace_bytes(0, ctypes.cast(arr, ctypes.c_void_p)) == 0
    arr = (P * 2)(good, good)
    plan = ctypes.c_void_p()
    bad_t = tsqr.BatchTuning(1000, 2048, 64)  # rows not a multiple of 64
    assert lib.tsqr_batched_create(0, 0, 2, ctypes.cast(arr, ctypes.c_void_p), 16, 1 << 30, 16,
                                   ctypes.byref(bad_t), ctypes.byref(plan)) == -8
    assert lib.tsqr_batched_create(0, 3, 2, ctypes.cast(arr, ctypes.c_void_p), 16, 1 << 30, 16,
                                   None, ctypes.byref(plan)) == -2  # precision
    assert lib.tsqr_batched_run(None, None) == -1
    assert lib.tsqr_batched_launches(None) == 0


def test_mixed_width_limit(lib):
    """The low-precision kernels stop at n = 256: no workspace size above."""
    assert lib.tsqr_mixed_workspace_bytes(4096, 256, 512, 1) > 0
    assert lib.tsqr_mixed_workspace_bytes(4096, 300, 600, 1) == 0
    assert lib.tsqr_workspace_bytes(4096, 1024, 2048) > 0


def test_rows_and_cholqr_argument_codes(lib):
    """Host-only argument checks of the row-extraction and CholeskyQR-family entries."""
    A, Q, R, W = (ctypes.c_void_p(x) for x in (0x10000000, 0x20000000, 0x30000000, 0x40000000))
    rows = lib.tsqr_rxr_cholqr_rows_ws
    assert rows(2, 64, 8, A, 64, 16, 1, 1, Q, 64, R, 8, W, 1, None, None) == -1   # variant
    assert rows(0, 64, 8, A, 64, 4, 1, 1, Q, 64, R, 8, W, 1, None, None) == -6    # s < n
    assert rows(0, 64, 8, A, 64, 16, 1, 1, Q, 64, R, 8, None, 1, None, None) == -13
    assert rows(0, 64, 8, A, 64, 16, 1, 1, Q, 64, R, 8, W, 1, None, None) == -101  # too small
    sk = lib.tsqr_sketch_rows
    assert sk(0, 8, A, 64, 16, 1, Q, 16, None) == -1
    assert sk(64, 0, A, 64, 16, 1, Q, 16, None) == -2
    assert sk(64, 8, None, 64, 16, 1, Q, 16, None) == -3
    assert sk(64, 8, A, 63, 16, 1, Q, 16, None) == -4
    assert sk(64, 8, A, 64, 0, 1, Q, 16, None) == -5
    assert sk(64, 8, A, 64, 16, 1, None, 16, None) == -7
    assert sk(64, 8, A, 64, 16, 1, Q, 15, None) == -8
    lib.tsqr_cholqr_workspace_bytes.restype = ctypes.c_size_t
    assert lib.tsqr_cholqr_workspace_bytes(64, 8) > 0
    assert lib.tsqr_cholqr_workspace_bytes(4, 8) == 0
    assert lib.tsqr_cholqr_workspace_bytes(4096, 2000) == 0
    ch = lib.tsqr_cholqr_ws
    ch.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                   ctypes.c_double, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                   ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                   ctypes.c_void_p]
    assert ch(4, 64, 8, A, 64, -1.0, Q, 64, R, 8, W, 1, None, None) == -1        # algo
    assert ch(2, 4, 8, A, 4, -1.0, Q, 4, R, 8, W, 1, None, None) == -2           # m < n
    assert ch(2, 64, 8, A, 63, -1.0, Q, 64, R, 8, W, 1, None, None) == -5        # lda
    assert ch(3, 64, 8, A, 64, float("nan"), Q, 64, R, 8, W, 1, None, None) == -6
    assert ch(2, 64, 8, A, 64, -1.0, A, 64, R, 8, W, 1, None, None) == -7        # Q aliases A
    assert ch(2, 64, 8, A, 64, -1.0, Q, 64, R, 8, None, 1, None, None) == -11
    assert ch(2, 64, 8, A, 64, -1.0, Q, 64, R, 8, W, 1, None, None) == -101      # too small


def test_lstsq_argument_codes(lib):
    A, b, x, W = (ctypes.c_void_p(v) for v in (0x10000000, 0x20000000, 0x30000000, 0x40000000))
    f = lib.tsqr_lstsq_ws
    lib.tsqr_lstsq_workspace_bytes.restype = ctypes.c_size_t
    assert lib.tsqr_lstsq_workspace_bytes(64, 8, 16) > 0
    assert lib.tsqr_lstsq_workspace_bytes(64, 8, 4) == 0
    assert f(2, 0, 64, 8, A, 64, b, 16, 1, x, W, 1, None, None) == -1    # variant
    assert f(0, 2, 64, 8, A, 64, b, 16, 1, x, W, 1, None, None) == -2    # sketch kind
    assert f(0, 0, 4, 8, A, 4, b, 16, 1, x, W, 1, None, None) == -3     # m < n
    assert f(0, 0, 64, 0, A, 64, b, 16, 1, x, W, 1, None, None) == -4   # n < 1
    assert f(0, 0, 64, 8, None, 64, b, 16, 1, x, W, 1, None, None) == -5
    assert f(0, 0, 64, 8, A, 63, b, 16, 1, x, W, 1, None, None) == -6
    assert f(0, 0, 64, 8, A, 64, None, 16, 1, x, W, 1, None, None) == -7
    assert f(0, 0, 64, 8, A, 64, b, 4, 1, x, W, 1, None, None) == -8
    assert f(0, 0, 64, 8, A, 64, b, 16, 1, None, W, 1, None, None) == -10
    assert f(0, 0, 64, 8, A, 64, b, 16, 1, x, None, 1, None, None) == -11
    assert f(0, 1, 64, 8, A, 64, b, 16, 1, x, W, 1, None, None) == -101  # workspace too small


def test_metrics_and_probe_argument_codes(lib):
    A = ctypes.c_void_p(0x10000000)
    Q = ctypes.c_void_p(0x20000000)
    R = ctypes.c_void_p(0x30000000)
    out = ctypes.c_void_p(0x40000000)
    W = ctypes.c_void_p(0x50000000)
    nb = lib.tsqr_metrics_workspace_bytes(1000, 40)
    assert nb > 0 and lib.tsqr_metrics_workspace_bytes(0, 4) == 0
    f = lib.tsqr_metrics
    assert f(0, 4, A, 8, Q, 8, R, 4, out, W, nb, None) == -1        # m < 1
    assert f(8, 0, A, 8, Q, 8, R, 4, out, W, nb, None) == -2        # n < 1
    assert f(8, 4, A, 7, Q, 8, R, 4, out, W, nb, None) == -4        # lda < m
    assert f(8, 4, A, 8, None, 8, R, 4, out, W, nb, None) == -5     # Q NULL
    assert f(8, 4, A, 8, Q, 7, R, 4, out, W, nb, None) == -6        # ldq < m
    assert f(8, 4, A, 8, Q, 8, R, 3, out, W, nb, None) == -8        # ldr < n
    assert f(8, 4, A, 8, Q, 8, R, 4, None, W, nb, None) == -9       # d_out NULL
    assert f(1000, 40, A, 1000, Q, 1000, R, 40, out, W, nb - 1, None) == -101  # workspace
    assert f(1000, 40, A, 1000, Q, 1000, R, 40, out, None, nb, None) == -101
    g = lib.tsqr_probe_stream
    assert g(3, A, Q, 1 << 20, 16, 4, 0, out, None) == -1
    assert g(0, None, Q, 1 << 20, 16, 4, 0, out, None) == -2
    assert g(1, A, None, 1 << 20, 16, 4, 0, out, None) == -3
    assert g(2, A, Q, 8, 16, 4, 0, out, None) == -4
    assert g(2, A, Q, 1 << 20, 0, 4, 0, out, None) == -5
    assert g(2, A, Q, 1 << 20, 16, 3, 0, out, None) == -6
    assert g(2, A, Q, 1 << 20, 16, 4, 0, None, None) == -8
    h = lib.tsqr_probe_mfma
    fl = ctypes.c_double()
    assert h(5, 2, 8, 10, out, ctypes.byref(fl), None) == -1  # kinds 0..4
    assert h(-1, 2, 8, 10, out, ctypes.byref(fl), None) == -1
    assert h(0, 3, 8, 10, out, ctypes.byref(fl), None) == -2
    assert h(0, 2, 5, 10, out, ctypes.byref(fl), None) == -3
    assert h(0, 2, 8, 0, out, ctypes.byref(fl), None) == -4
    assert h(0, 2, 8, 10, None, ctypes.byref(fl), None) == -5
    assert h(0, 2, 8, 10, out, None, None) == -6


def test_noalloc_refuses_sizes_beyond_the_array(lib):
    # refused before any work is enqueued: a workspace above the fixed per-GPU array
    assert lib.tsqr_workspace_bytes(1 << 20, 256, 512) > (72 << 20)
    assert lib.tsqr_workspace_bytes(1 << 24, 128, 256) <= (72 << 20)
    A = ctypes.c_void_p(0x10000000)
    Q = ctypes.c_void_p(0x7000000000)
    f = lib.tsqr_rxr_cholqr_noalloc
    assert f(0, 1 << 20, 256, A, 1 << 20, 512, 1, 1, Q, 1 << 20, None, 256, None, None) == -101
    assert f(2, 1 << 20, 128, A, 1 << 20, 256, 1, 1, Q, 1 << 20, None, 128, None, None) == -1
    assert f(0, 1 << 20, 128, A, 1 << 20, 100, 1, 1, Q, 1 << 20, None, 128, None, None) == -6
