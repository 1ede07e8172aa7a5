"""NumPy front end of the FP64 CPU oracle (``oracle/tsqr_oracle.c``).

Test infrastructure only: the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` are the only callers.  The GPU library never imports this module.

Every matrix argument is a float64 NumPy array in Fortran (column-major) order; the
wrappers pass pointers and leading dimensions straight through to the C routines.
The C library is built by ``oracle/build.py`` (called from ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_c_i64 = ctypes.c_int64
_c_u64 = ctypes.c_uint64
_c_dp = ctypes.POINTER(ctypes.c_double)
_c_int = ctypes.c_int

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _b  # noqa: F401  (build on first use)

        _b.build()
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "or_philox4x32_10": (None, [ctypes.POINTER(ctypes.c_uint32)] * 3),
        "or_philox4x64_10": (None, [ctypes.POINTER(ctypes.c_uint64)] * 3),
        "or_sketch_normal": (ctypes.c_double, [_c_u64, _c_i64, _c_i64]),
        "or_sketch_normals": (None, [_c_u64, _c_i64, _c_i64, _c_i64, _c_i64, _c_dp, _c_i64]),
        "or_sketch_apply": (None, [_c_i64, _c_i64, _c_dp, _c_i64, _c_i64, _c_u64, _c_dp, _c_i64]),
        "or_householder_r": (_c_int, [_c_i64, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64]),
        "or_lu_r": (_c_int, [_c_i64, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64,
                             ctypes.POINTER(ctypes.c_int64)]),
        "or_trsm_ru": (None, [_c_i64, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64]),
        "or_gram": (None, [_c_i64, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64]),
        "or_cholesky_upper": (_c_int, [_c_i64, _c_dp, _c_i64, _c_dp, _c_i64]),
        "or_trmm_upper": (None, [_c_i64, _c_dp, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64]),
        "or_rxr_cholqr": (_c_int, [_c_int, _c_i64, _c_i64, _c_dp, _c_i64, _c_i64, _c_u64,
                                   _c_int, _c_dp, _c_i64, _c_dp, _c_i64, _c_dp, _c_dp,
                                   _c_dp]),
        "or_rxr_cholqr_rows": (_c_int, [_c_int, _c_i64, _c_i64, _c_dp, _c_i64, _c_i64,
                                        _c_u64, _c_int, _c_dp, _c_i64, _c_dp, _c_i64, _c_dp,
                                        _c_dp, _c_dp]),
        "or_sample_rows": (None, [_c_i64, _c_i64, _c_u64, ctypes.POINTER(ctypes.c_int64)]),
        "or_lstsq_rxr": (_c_int, [_c_int, _c_int, _c_i64, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64,
                                  _c_u64, _c_dp]),
        "or_sketch_rows": (None, [_c_i64, _c_i64, _c_dp, _c_i64, _c_i64, _c_u64, _c_dp,
                                  _c_i64]),
        "or_cholqr_n": (_c_int, [_c_i64, _c_i64, _c_dp, _c_i64, _c_int, ctypes.c_double,
                                 _c_dp, _c_i64, _c_dp, _c_i64]),
        "or_orthogonality": (ctypes.c_double, [_c_i64, _c_i64, _c_dp, _c_i64]),
        "or_residual": (ctypes.c_double, [_c_i64, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64,
                                          _c_dp, _c_i64]),
        "or_num_threads": (_c_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(x: np.ndarray, name: str) -> np.ndarray:
    if x.dtype != np.float64:
        raise TypeError(f"{name}: expected float64, got {x.dtype}")
    if x.ndim != 2:
        raise ValueError(f"{name}: expected a matrix")
    if not x.flags.f_contiguous:
        raise ValueError(f"{name}: expected a column-major (Fortran-ordered) array")
    return x


def _ptr(x: np.ndarray):
    return x.ctypes.data_as(_c_dp)


def _ld(x: np.ndarray) -> int:
    return max(1, x.shape[0])


# ---------------------------------------------------------------------------- RNG ----
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    p = ctypes.POINTER(ctypes.c_uint32)
    _load().or_philox4x32_10(c.ctypes.data_as(p), k.ctypes.data_as(p), out.ctypes.data_as(p))
    return out


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    p = ctypes.POINTER(ctypes.c_uint64)
    _load().or_philox4x64_10(c.ctypes.data_as(p), k.ctypes.data_as(p), out.ctypes.data_as(p))
    return out


def sketch_normal(seed: int, i: int, j: int) -> float:
    return _load().or_sketch_normal(seed, i, j)


def sketch_normals(seed: int, i0: int, ni: int, j0: int, nj: int) -> np.ndarray:
    """Z(i0:i0+ni, j0:j0+nj), the N(0,1) entries of the sketch before the 1/sqrt(s)."""
    Z = np.zeros((ni, nj), dtype=np.float64, order="F")
    _load().or_sketch_normals(seed, i0, ni, j0, nj, _ptr(Z), max(1, ni))
    return Z


# -------------------------------------------------------------------------- steps ----
def sketch_apply(A: np.ndarray, s: int, seed: int) -> np.ndarray:
    A = _f64(A, "A")
    m, n = A.shape
    B = np.zeros((s, n), dtype=np.float64, order="F")
    _load().or_sketch_apply(m, n, _ptr(A), _ld(A), s, seed, _ptr(B), max(1, s))
    return B


def householder_r(B: np.ndarray):
    B = _f64(B, "B")
    s, n = B.shape
    R = np.zeros((n, n), dtype=np.float64, order="F")
    info = _load().or_householder_r(s, n, _ptr(B), _ld(B), _ptr(R), max(1, n))
    return R, info


def lu_r(B: np.ndarray):
    B = _f64(B, "B")
    s, n = B.shape
    R = np.zeros((n, n), dtype=np.float64, order="F")
    piv = np.zeros(max(1, n), dtype=np.int64)
    info = _load().or_lu_r(s, n, _ptr(B), _ld(B), _ptr(R), max(1, n),
                           piv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return R, piv[:n], info


def trsm_ru(Y: np.ndarray, T: np.ndarray) -> np.ndarray:
    Y = _f64(Y, "Y")
    T = _f64(T, "T")
    m, n = Y.shape
    X = np.zeros((m, n), dtype=np.float64, order="F")
    _load().or_trsm_ru(m, n, _ptr(Y), _ld(Y), _ptr(T), _ld(T), _ptr(X), max(1, m))
    return X


def gram(X: np.ndarray) -> np.ndarray:
    X = _f64(X, "X")
    m, n = X.shape
    W = np.zeros((n, n), dtype=np.float64, order="F")
    _load().or_gram(m, n, _ptr(X), _ld(X), _ptr(W), max(1, n))
    return W


def cholesky_upper(W: np.ndarray):
    W = _f64(W, "W")
    n = W.shape[0]
    R = np.zeros((n, n), dtype=np.float64, order="F")
    info = _load().or_cholesky_upper(n, _ptr(W), _ld(W), _ptr(R), max(1, n))
    return R, info


def trmm_upper(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    A = _f64(A, "A")
    B = _f64(B, "B")
    n = A.shape[0]
    C = np.zeros((n, n), dtype=np.float64, order="F")
    _load().or_trmm_upper(n, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C), max(1, n))
    return C


# ------------------------------------------------------------------------ drivers ----
RQR = 0
RLU = 1


def rxr_cholqr(A: np.ndarray, s: int, seed: int, variant: int = RQR, extra_pass: bool = True,
               sketch: str = "gaussian"):
    """Randomized XR-preconditioned CholeskyQR with the Gaussian (default) or the
    row-extraction sketch.  Returns dict(Q, R, R0, R1, R2, info)."""
    A = _f64(A, "A")
    m, n = A.shape
    Q = np.zeros((m, n), dtype=np.float64, order="F")
    R = np.zeros((n, n), dtype=np.float64, order="F")
    R0 = np.zeros((n, n), dtype=np.float64, order="F")
    R1 = np.zeros((n, n), dtype=np.float64, order="F")
    R2 = np.zeros((n, n), dtype=np.float64, order="F")
    if sketch not in ("gaussian", "rows"):
        raise ValueError(f"unknown sketch {sketch!r}")
    fn = _load().or_rxr_cholqr if sketch == "gaussian" else _load().or_rxr_cholqr_rows
    info = fn(variant, m, n, _ptr(A), _ld(A), s, seed, int(extra_pass), _ptr(Q), max(1, m),
              _ptr(R), max(1, n), _ptr(R0), _ptr(R1), _ptr(R2))
    return {"Q": Q, "R": R, "R0": R0, "R1": R1, "R2": R2, "info": info}


def lstsq(A: np.ndarray, b: np.ndarray, s: int, seed: int, variant: int = RQR,
          sketch: str = "gaussian"):
    """Least squares preconditioned by the sketch's R factor (Section 5.2).
    Returns (x, info)."""
    A = _f64(A, "A")
    m, n = A.shape
    b = np.ascontiguousarray(b, dtype=np.float64).reshape(m)
    x = np.zeros(n, dtype=np.float64)
    info = _load().or_lstsq_rxr(variant, 0 if sketch == "gaussian" else 1, m, n, _ptr(A),
                                _ld(A), b.ctypes.data_as(_c_dp), s, seed,
                                x.ctypes.data_as(_c_dp))
    return x, info


def sample_rows(m: int, s: int, seed: int) -> np.ndarray:
    """Row indices r_0..r_{s-1} of the row-extraction sketch (int64)."""
    rows = np.zeros(s, dtype=np.int64)
    _load().or_sample_rows(m, s, seed, rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return rows


def sketch_rows(A: np.ndarray, s: int, seed: int) -> np.ndarray:
    """B = A(rows, :) of the row-extraction sketch."""
    A = _f64(A, "A")
    m, n = A.shape
    B = np.zeros((s, n), dtype=np.float64, order="F")
    _load().or_sketch_rows(m, n, _ptr(A), _ld(A), s, seed, _ptr(B), max(1, s))
    return B


def cholqr_n(A: np.ndarray, npass: int, shift: float = 0.0):
    """CholeskyQR (npass=1), CholeskyQR2 (npass=2), shifted CholeskyQR3 (npass=3, shift != 0;
    shift < 0 = the paper's suggested 11(mn + n(n+1)) u ||A||_2^2, bounded by ||A^T A||_F)."""
    A = _f64(A, "A")
    m, n = A.shape
    Q = np.zeros((m, n), dtype=np.float64, order="F")
    R = np.zeros((n, n), dtype=np.float64, order="F")
    info = _load().or_cholqr_n(m, n, _ptr(A), _ld(A), npass, shift, _ptr(Q), max(1, m),
                               _ptr(R), max(1, n))
    return Q, R, info


# ------------------------------------------------------------------------ metrics ----
def orthogonality(Q: np.ndarray) -> float:
    """||Q^T Q - I||_F with double-double accumulation."""
    Q = _f64(Q, "Q")
    m, n = Q.shape
    return _load().or_orthogonality(m, n, _ptr(Q), _ld(Q))


def residual(A: np.ndarray, Q: np.ndarray, R: np.ndarray) -> float:
    """||A - Q R||_F / ||A||_F with double-double accumulation."""
    A = _f64(A, "A")
    Q = _f64(Q, "Q")
    R = _f64(R, "R")
    m, n = A.shape
    return _load().or_residual(m, n, _ptr(A), _ld(A), _ptr(Q), _ld(Q), _ptr(R), _ld(R))


def num_threads() -> int:
    return _load().or_num_threads()


# ------------------------------------------------------------------ mixed precision ----
FP32 = 1
BF16 = 2

_MIXED_SIGS = {
    "or_round_fp32": (ctypes.c_double, [ctypes.c_double]),
    "or_round_bf16": (ctypes.c_double, [ctypes.c_double]),
    "or_sketch_apply_lowp": (None, [_c_int, _c_i64, _c_i64, _c_dp, _c_i64, _c_i64, _c_u64, _c_dp,
                                    _c_i64]),
    "or_apply_rinv_lowp": (None, [_c_int, _c_i64, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64, _c_dp,
                                  _c_i64]),
    "or_gram_lowp": (None, [_c_int, _c_i64, _c_i64, _c_dp, _c_i64, _c_dp, _c_i64]),
    "or_trtri_upper": (None, [_c_i64, _c_dp, _c_i64, _c_dp, _c_i64]),
    "or_rxr_cholqr_mixed": (_c_int, [_c_int, _c_int, _c_i64, _c_i64, _c_dp, _c_i64, _c_i64, _c_u64,
                                     _c_int, _c_dp, _c_i64, _c_dp, _c_i64,
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
}


def _load_mixed():
    lib = _load()
    if not getattr(lib, "_mixed_sigs", False):
        for name, (res, args) in _MIXED_SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        lib._mixed_sigs = True
    return lib


def round_fp32(x: float) -> float:
    return _load_mixed().or_round_fp32(x)


def round_bf16(x: float) -> float:
    return _load_mixed().or_round_bf16(x)


def sketch_apply_lowp(prec: int, A: np.ndarray, s: int, seed: int) -> np.ndarray:
    A = _f64(A, "A")
    m, n = A.shape
    B = np.zeros((s, n), dtype=np.float64, order="F")
    _load_mixed().or_sketch_apply_lowp(prec, m, n, _ptr(A), _ld(A), s, seed, _ptr(B), max(1, s))
    return B


def apply_rinv_lowp(prec: int, Y: np.ndarray, Rinv: np.ndarray) -> np.ndarray:
    Y = _f64(Y, "Y")
    Rinv = _f64(Rinv, "Rinv")
    m, n = Y.shape
    X = np.zeros((m, n), dtype=np.float64, order="F")
    _load_mixed().or_apply_rinv_lowp(prec, m, n, _ptr(Y), _ld(Y), _ptr(Rinv), _ld(Rinv), _ptr(X),
                                     max(1, m))
    return X


def gram_lowp(prec: int, X: np.ndarray) -> np.ndarray:
    X = _f64(X, "X")
    m, n = X.shape
    W = np.zeros((n, n), dtype=np.float64, order="F")
    _load_mixed().or_gram_lowp(prec, m, n, _ptr(X), _ld(X), _ptr(W), max(1, n))
    return W


def trtri_upper(T: np.ndarray) -> np.ndarray:
    T = _f64(T, "T")
    n = T.shape[0]
    X = np.zeros((n, n), dtype=np.float64, order="F")
    _load_mixed().or_trtri_upper(n, _ptr(T), _ld(T), _ptr(X), max(1, n))
    return X


def rxr_cholqr_mixed(A: np.ndarray, s: int, seed: int, prec: int = FP32, variant: int = RQR,
                     fp64_passes: int = 1):
    A = _f64(A, "A")
    m, n = A.shape
    Q = np.zeros((m, n), dtype=np.float64, order="F")
    R = np.zeros((n, n), dtype=np.float64, order="F")
    lp = ctypes.c_int(0)
    npass = ctypes.c_int(0)
    info = _load_mixed().or_rxr_cholqr_mixed(variant, prec, m, n, _ptr(A), _ld(A), s, seed,
                                             fp64_passes, _ptr(Q), max(1, m), _ptr(R), max(1, n),
                                             ctypes.byref(lp), ctypes.byref(npass))
    return {"Q": Q, "R": R, "info": info, "lp_info": lp.value, "passes": npass.value}
