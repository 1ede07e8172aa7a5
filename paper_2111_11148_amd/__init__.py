"""Randomized XR-preconditioned CholeskyQR on AMD Instinct MI355X (gfx950).

Thin Python binding of ``libtsqr.so`` (C ABI in ``include/tsqr.h``).  Every function here
only marshals arguments: it checks dtypes, devices and column-major strides of torch
tensors and passes their device pointers and the current HIP stream to the library.
All arithmetic runs in the library's HIP kernels; there is no fallback path, and a
missing or unloadable library raises.

Matrices are column-major: an m x n matrix is a float64 CUDA tensor of shape (m, n) with
strides (1, ld), ld >= m (see :func:`colmajor`).
"""
from __future__ import annotations

import contextlib
import ctypes
import functools
import inspect
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsqr.so")

RQR = 0
RLU = 1
TSQR_ERR_HIP = -100
TSQR_ERR_WORKSPACE = -101
TSQR_ERR_UNSUPPORTED = -102

_lib = None

_i64, _u64, _int, _vp, _sz = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p,
                              ctypes.c_size_t)
_SIGS = {
    "tsqr_rqr_cholqr": (_int, [_i64, _i64, _vp, _i64, _i64, _u64, _vp, _vp, _vp]),
    "tsqr_rlu_cholqr": (_int, [_i64, _i64, _vp, _i64, _i64, _u64, _vp, _vp, _vp]),
    "tsqr_workspace_bytes": (_sz, [_i64, _i64, _i64]),
    "tsqr_rxr_cholqr_ws": (_int, [_int, _i64, _i64, _vp, _i64, _i64, _u64, _int, _vp, _i64, _vp,
                                  _i64, _vp, _sz, _vp, _vp]),
    "tsqr_rxr_cholqr_noalloc": (_int, [_int, _i64, _i64, _vp, _i64, _i64, _u64, _int, _vp, _i64,
                                       _vp, _i64, _vp, _vp]),
    "tsqr_rxr_cholqr_rows_ws": (_int, [_int, _i64, _i64, _vp, _i64, _i64, _u64, _int, _vp, _i64,
                                       _vp, _i64, _vp, _sz, _vp, _vp]),
    "tsqr_sketch_rows": (_int, [_i64, _i64, _vp, _i64, _i64, _u64, _vp, _i64, _vp]),
    "tsqr_cholqr_workspace_bytes": (_sz, [_i64, _i64]),
    "tsqr_lstsq_workspace_bytes": (_sz, [_i64, _i64, _i64]),
    "tsqr_lstsq_ws": (_int, [_int, _int, _i64, _i64, _vp, _i64, _vp, _i64, _u64, _vp, _vp, _sz,
                             _vp, _vp]),
    "tsqr_cholqr_ws": (_int, [_int, _i64, _i64, _vp, _i64, ctypes.c_double, _vp, _i64, _vp,
                              _i64, _vp, _sz, _vp, _vp]),
    "tsqr_sketch_workspace_bytes": (_sz, [_i64, _i64, _i64]),
    "tsqr_sketch": (_int, [_i64, _i64, _vp, _i64, _i64, _u64, _vp, _i64, _vp, _sz, _vp]),
    "tsqr_sketch_factor_workspace_bytes": (_sz, [_i64, _i64]),
    "tsqr_sketch_factor": (_int, [_int, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _sz, _vp]),
    "tsqr_trsm_workspace_bytes": (_sz, [_i64]),
    "tsqr_trsm": (_int, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp]),
    "tsqr_gram_workspace_bytes": (_sz, [_i64, _i64]),
    "tsqr_gram": (_int, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp]),
    "tsqr_potrf": (_int, [_i64, _vp, _i64, _vp, _i64, _int, _vp, _vp, _sz, _vp]),
    "tsqr_trmm_upper": (_int, [_i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp]),
    "tsqr_philox4x32_10": (_int, [_i64, _vp, _u64, _vp, _vp]),
    "tsqr_sketch_normals": (_int, [_u64, _i64, _i64, _i64, _i64, _vp, _i64, _vp]),
    "tsqr_version": (ctypes.c_char_p, []),
    "tsqr_mixed_workspace_bytes": (_sz, [_i64, _i64, _i64, _int]),
    "tsqr_rxr_cholqr_mixed_ws": (_int, [_int, _int, _i64, _i64, _vp, _i64, _i64, _u64, _int, _vp,
                                        _i64, _vp, _i64, _vp, _sz, _vp, _vp, _vp]),
    "tsqr_sketch_lowp": (_int, [_int, _i64, _i64, _vp, _i64, _i64, _u64, _vp, _i64, _vp, _sz, _vp]),
    "tsqr_rinv_lowp_bytes": (_sz, [_i64, _int]),
    "tsqr_apply_rinv_lowp": (_int, [_int, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _sz,
                                    _vp]),
    "tsqr_gram_lowp": (_int, [_int, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp]),
    "tsqr_batched_workspace_bytes": (_sz, [_i64, _vp]),
    "tsqr_batched_create": (_int, [_int, _int, _i64, _vp, _vp, _sz, _vp, _vp,
                                   ctypes.POINTER(_vp)]),
    "tsqr_batched_autotune": (_int, [_int, _int, _i64, _vp, _vp, _sz, _vp, _vp, _vp,
                                     ctypes.POINTER(ctypes.c_double)]),
    "tsqr_batched_autotune_persistent": (_int, [_int, _int, _i64, _vp, _vp, _sz, _vp, _vp, _vp,
                                     ctypes.POINTER(ctypes.c_double)]),
    "tsqr_batched_run": (_int, [_vp, _vp]),
    "tsqr_batched_run_persistent": (_int, [_vp, _vp]),
    "tsqr_batched_run_persistent_timed": (_int, [_vp, _vp, _vp]),
    "tsqr_batched_launches": (_int, [_vp]),
    "tsqr_batched_tasks": (_int, [_vp]),
    "tsqr_batched_destroy": (None, [_vp]),
    "tsqr_metrics_workspace_bytes": (_sz, [_i64, _i64]),
    "tsqr_metrics": (_int, [_i64, _i64, _vp, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _sz, _vp]),
    "tsqr_probe_stream": (_int, [_int, _vp, _vp, _sz, _int, _int, _int, _vp, _vp]),
    "tsqr_probe_mfma": (_int, [_int, _int, _int, _i64, _vp, ctypes.POINTER(ctypes.c_double),
                               _vp]),
    "tsqr_profile_start": (_int, []),
    "tsqr_profile_only": (_int, [ctypes.c_char_p]),
    "tsqr_profile_stop": (_int, []),
    "tsqr_profile_record": (_int, [_int, ctypes.POINTER(ctypes.c_char_p),
                                   ctypes.POINTER(ctypes.c_double)]),
}


class TsqrError(RuntimeError):
    """A libtsqr call returned a nonzero status."""


def load() -> ctypes.CDLL:
    """Load libtsqr.so (built by ``paper_2111_11148_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def version() -> str:
    return load().tsqr_version().decode()


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise TsqrError(f"{what} failed with status {rc}")


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _on_stream(fn):
    """Run `fn` with its `stream` argument (when given) as torch's current stream, so that
    every tensor it allocates (outputs, workspace, info) comes from that stream's pool of
    the caching allocator: a temporary freed on return is then not handed to work on
    another stream while this call's kernels still use it."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapper(*args, **kwargs):
        stream = sig.bind(*args, **kwargs).arguments.get("stream")
        ctx = torch.cuda.stream(stream) if stream is not None else contextlib.nullcontext()
        with ctx:
            return fn(*args, **kwargs)
    return wrapper


def _mat(t: torch.Tensor, name: str, rows: int | None = None, cols: int | None = None) -> int:
    """Validate a column-major FP64 device matrix; return its leading dimension."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name}: expected float64, got {t.dtype}")
    if t.device.type != "cuda":
        raise ValueError(f"{name}: expected a GPU tensor")
    if t.dim() != 2:
        raise ValueError(f"{name}: expected a matrix")
    if rows is not None and t.shape[0] != rows or cols is not None and t.shape[1] != cols:
        raise ValueError(f"{name}: expected shape ({rows}, {cols}), got {tuple(t.shape)}")
    r, c = t.shape
    if c > 1 and r > 1 and t.stride(0) != 1:
        raise ValueError(f"{name}: expected column-major strides (1, ld)")
    ld = t.stride(1) if c > 1 else max(r, 1)
    if ld < r:
        raise ValueError(f"{name}: leading dimension {ld} < rows {r}")
    return int(ld)


def colmajor(m: int, n: int, ld: int | None = None, device="cuda", dtype=torch.float64,
             fill=None) -> torch.Tensor:
    """Uninitialised (or filled) m x n column-major tensor with leading dimension ld."""
    ld = m if ld is None else ld
    buf = torch.empty((n, ld), device=device, dtype=dtype)
    if fill is not None:
        buf.fill_(fill)
    return buf.t()[:m]


def to_device_colmajor(A, ld: int | None = None, device="cuda") -> torch.Tensor:
    """Copy a host matrix (NumPy or torch) into a column-major device tensor."""
    At = torch.as_tensor(A, dtype=torch.float64)
    m, n = At.shape
    out = colmajor(m, n, ld, device=device)
    out.copy_(At)
    return out


# ------------------------------------------------------------------ phase timing ----
def profile_start(only: str | None = None) -> None:
    """Start recording phase events; `only` limits them to the phase of that name."""
    _check(load().tsqr_profile_only(only.encode() if only else None), "tsqr_profile_only")
    _check(load().tsqr_profile_start(), "tsqr_profile_start")


def profile_stop():
    """Stop recording; return [(phase name, milliseconds), ...] in launch order."""
    lib = load()
    count = lib.tsqr_profile_stop()
    if count < 0:
        raise TsqrError(f"tsqr_profile_stop failed with status {count}")
    out = []
    name = ctypes.c_char_p()
    ms = ctypes.c_double()
    for i in range(count):
        _check(lib.tsqr_profile_record(i, ctypes.byref(name), ctypes.byref(ms)),
               "tsqr_profile_record")
        out.append((name.value.decode(), ms.value))
    return out


# ------------------------------------------------------- accuracy metrics, probes ----
@_on_stream
def metrics(Q: torch.Tensor, A: torch.Tensor | None = None, R: torch.Tensor | None = None,
            stream=None):
    """(||Q^T Q - I||_F, ||A - Q R||_F / ||A||_F) with double-double accumulation on the
    device; the residual is NaN when A or R is not given.  Returns two Python floats."""
    ldq = _mat(Q, "Q")
    m, n = Q.shape
    lda = _mat(A, "A", m, n) if A is not None else m
    ldr = _mat(R, "R", n, n) if R is not None else n
    lib = load()
    work = torch.empty(max(1, int(lib.tsqr_metrics_workspace_bytes(m, n))), dtype=torch.uint8,
                       device=Q.device)
    out = torch.empty(2, dtype=torch.float64, device=Q.device)
    rc = lib.tsqr_metrics(m, n, A.data_ptr() if A is not None else None, lda, Q.data_ptr(), ldq,
                          R.data_ptr() if R is not None else None, ldr, out.data_ptr(),
                          work.data_ptr(), work.numel(), _stream(stream))
    _check(rc, "tsqr_metrics")
    o = out.cpu()
    return float(o[0]), float(o[1])


PROBE_READ, PROBE_WRITE, PROBE_COPY = 0, 1, 2
PROBE_FP64, PROBE_FP32, PROBE_BF16, PROBE_BF16_32, PROBE_FP64_RANDOM = 0, 1, 2, 3, 4


def probe_stream(kind: int, src: torch.Tensor | None, dst: torch.Tensor | None, nbytes: int,
                 sink: torch.Tensor, wgs_per_cu: int = 16, unroll: int = 4,
                 nontemporal: bool = False, stream=None) -> None:
    """One pass of the streaming probe (read / write / copy of nbytes)."""
    rc = load().tsqr_probe_stream(kind, src.data_ptr() if src is not None else None,
                                  dst.data_ptr() if dst is not None else None, nbytes,
                                  wgs_per_cu, unroll, int(bool(nontemporal)), sink.data_ptr(),
                                  _stream(stream))
    _check(rc, "tsqr_probe_stream")


def probe_mfma(kind: int, iters: int, sink: torch.Tensor, waves_per_simd: int = 2,
               chains: int = 8, stream=None) -> float:
    """One launch of the matrix-core probe; returns its flop count."""
    fl = ctypes.c_double()
    rc = load().tsqr_probe_mfma(kind, waves_per_simd, chains, iters, sink.data_ptr(),
                                ctypes.byref(fl), _stream(stream))
    _check(rc, "tsqr_probe_mfma")
    return fl.value


# ------------------------------------------------------------------ whole method ----
def workspace_bytes(m: int, n: int, sketch_rows: int) -> int:
    return int(load().tsqr_workspace_bytes(m, n, sketch_rows))


def alloc_workspace(m: int, n: int, sketch_rows: int, device="cuda") -> torch.Tensor:
    nbytes = workspace_bytes(m, n, sketch_rows)
    if nbytes == 0:
        raise ValueError("invalid sizes for the workspace")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


@_on_stream
def rxr_cholqr(A: torch.Tensor, sketch_rows: int, seed: int, variant: int = RQR,
               extra_pass: bool = True, Q: torch.Tensor | None = None,
               R: torch.Tensor | None = None, want_r: bool = True,
               workspace: torch.Tensor | None = None, info: torch.Tensor | None = None,
               stream=None, sketch: str = "gaussian"):
    """Randomized XR-preconditioned CholeskyQR (explicit-workspace entry point), with the
    Gaussian sketch (default) or the row-extraction sketch (``sketch="rows"``).

    Returns (Q, R, info) with info a 1-element int32 device tensor (0 = success)."""
    if sketch not in ("gaussian", "rows"):
        raise ValueError(f"unknown sketch {sketch!r}")
    lda = _mat(A, "A")
    m, n = A.shape
    if Q is None:
        Q = colmajor(m, n, device=A.device)
    ldq = _mat(Q, "Q", m, n)
    if R is None and want_r:
        R = colmajor(n, n, device=A.device)
    ldr = _mat(R, "R", n, n) if R is not None else n
    if workspace is None:
        workspace = alloc_workspace(m, n, sketch_rows, device=A.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    name = "tsqr_rxr_cholqr_ws" if sketch == "gaussian" else "tsqr_rxr_cholqr_rows_ws"
    rc = getattr(load(), name)(variant, m, n, A.data_ptr(), lda, sketch_rows, seed,
                               int(bool(extra_pass)), Q.data_ptr(), ldq,
                               R.data_ptr() if R is not None else None, ldr,
                               workspace.data_ptr(), workspace.numel(), info.data_ptr(),
                               _stream(stream))
    _check(rc, name)
    return Q, R, info


STATIC_SCRATCH_BYTES = 72 << 20


def rxr_cholqr_noalloc(A: torch.Tensor, sketch_rows: int, seed: int, Q: torch.Tensor,
                       R: torch.Tensor | None, info: torch.Tensor | None, variant: int = RQR,
                       extra_pass: bool = True, stream=None):
    """The no-allocation entry point: the library's fixed per-GPU scratch array serves as
    the workspace; every output (Q, R, info) is the caller's, and this call allocates
    nothing.  Calls that overlap in time on one GPU race.  Returns (Q, R, info)."""
    lda = _mat(A, "A")
    m, n = A.shape
    ldq = _mat(Q, "Q", m, n)
    ldr = _mat(R, "R", n, n) if R is not None else n
    rc = load().tsqr_rxr_cholqr_noalloc(variant, m, n, A.data_ptr(), lda, sketch_rows, seed,
                                        int(bool(extra_pass)), Q.data_ptr(), ldq,
                                        R.data_ptr() if R is not None else None, ldr,
                                        info.data_ptr() if info is not None else None,
                                        _stream(stream))
    _check(rc, "tsqr_rxr_cholqr_noalloc")
    return Q, R, info


CHOLQR = 1
CHOLQR2 = 2
SCHOLQR3 = 3


@_on_stream
def lstsq(A: torch.Tensor, b: torch.Tensor, sketch_rows: int, seed: int, variant: int = RQR,
          sketch: str = "gaussian", x: torch.Tensor | None = None,
          workspace: torch.Tensor | None = None, info: torch.Tensor | None = None, stream=None):
    """min ||A x - b||_2 preconditioned by the sketch's R factor.  Returns (x, info)."""
    lda = _mat(A, "A")
    m, n = A.shape
    if b.dtype != torch.float64 or b.device != A.device or b.shape != (m,) or b.stride() != (1,):
        raise ValueError("b must be a contiguous float64 vector of m entries on A's device")
    if x is None:
        x = torch.empty(n, dtype=torch.float64, device=A.device)
    if x.dtype != torch.float64 or x.shape != (n,) or x.stride() != (1,):
        raise ValueError("x must be a contiguous float64 vector of n entries")
    if workspace is None:
        workspace = torch.empty(max(1, int(load().tsqr_lstsq_workspace_bytes(m, n, sketch_rows))),
                                dtype=torch.uint8, device=A.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    kind = {"gaussian": 0, "rows": 1}[sketch]
    rc = load().tsqr_lstsq_ws(variant, kind, m, n, A.data_ptr(), lda, b.data_ptr(), sketch_rows,
                              seed, x.data_ptr(), workspace.data_ptr(), workspace.numel(),
                              info.data_ptr(), _stream(stream))
    _check(rc, "tsqr_lstsq_ws")
    return x, info


def cholqr_workspace_bytes(m: int, n: int) -> int:
    return int(load().tsqr_cholqr_workspace_bytes(m, n))


@_on_stream
def cholqr(A: torch.Tensor, algo: int = CHOLQR2, shift: float = -1.0,
           Q: torch.Tensor | None = None, R: torch.Tensor | None = None, want_r: bool = True,
           workspace: torch.Tensor | None = None, info: torch.Tensor | None = None,
           stream=None):
    """CholeskyQR (algo=CHOLQR), CholeskyQR2 or shifted CholeskyQR3 (shift < 0: the
    suggested 11(mn + n(n+1)) u ||A||_2^2 bound; >= 0: that shift).  Returns (Q, R, info)."""
    lda = _mat(A, "A")
    m, n = A.shape
    if Q is None:
        Q = colmajor(m, n, device=A.device)
    ldq = _mat(Q, "Q", m, n)
    if R is None and want_r:
        R = colmajor(n, n, device=A.device)
    ldr = _mat(R, "R", n, n) if R is not None else n
    if workspace is None:
        workspace = torch.empty(max(1, cholqr_workspace_bytes(m, n)), dtype=torch.uint8,
                                device=A.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    rc = load().tsqr_cholqr_ws(algo, m, n, A.data_ptr(), lda, float(shift), Q.data_ptr(), ldq,
                               R.data_ptr() if R is not None else None, ldr,
                               workspace.data_ptr(), workspace.numel(), info.data_ptr(),
                               _stream(stream))
    _check(rc, "tsqr_cholqr_ws")
    return Q, R, info


FP32 = 1
BF16 = 2


def mixed_workspace_bytes(m: int, n: int, sketch_rows: int, lowp: int) -> int:
    return int(load().tsqr_mixed_workspace_bytes(m, n, sketch_rows, lowp))


@_on_stream
def rxr_cholqr_mixed(A: torch.Tensor, sketch_rows: int, seed: int, lowp: int = FP32,
                     variant: int = RQR, fp64_passes: int = 0, Q: torch.Tensor | None = None,
                     R: torch.Tensor | None = None, want_r: bool = True,
                     workspace: torch.Tensor | None = None, info: torch.Tensor | None = None,
                     report: torch.Tensor | None = None, stream=None):
    """Mixed-precision variant: the sketch on `lowp` (FP32 or BF16) matrix cores, the
    preconditioner apply and first Gram matrix with FP32 inputs, FP64 passes.

    fp64_passes: 1-3 fixed FP64 CholeskyQR passes, or 0 for the automatic rule (decided on
    the device: the call never waits, so it may be captured into a graph).
    Returns (Q, R, info, report): info a 1-element int32 device tensor, report a
    2-element one holding the number of FP64 passes run and whether the low-precision
    stage ran (1) or was skipped (0)."""
    lda = _mat(A, "A")
    m, n = A.shape
    if Q is None:
        Q = colmajor(m, n, device=A.device)
    ldq = _mat(Q, "Q", m, n)
    if R is None and want_r:
        R = colmajor(n, n, device=A.device)
    ldr = _mat(R, "R", n, n) if R is not None else n
    if workspace is None:
        nbytes = mixed_workspace_bytes(m, n, sketch_rows, lowp)
        if nbytes == 0:
            raise ValueError("invalid sizes for the workspace")
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=A.device)
    if report is None:
        report = torch.zeros(2, dtype=torch.int32, device=A.device)
    rc = load().tsqr_rxr_cholqr_mixed_ws(variant, lowp, m, n, A.data_ptr(), lda, sketch_rows,
                                         seed, fp64_passes, Q.data_ptr(), ldq,
                                         R.data_ptr() if R is not None else None, ldr,
                                         workspace.data_ptr(), workspace.numel(),
                                         info.data_ptr(), report.data_ptr(), _stream(stream))
    _check(rc, "tsqr_rxr_cholqr_mixed_ws")
    return Q, R, info, report


@_on_stream
def sketch_lowp(A: torch.Tensor, s: int, seed: int, lowp: int = FP32, stream=None):
    lda = _mat(A, "A")
    m, n = A.shape
    B = colmajor(s, n, device=A.device)
    nbytes = int(load().tsqr_sketch_workspace_bytes(m, n, s))
    work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=A.device)
    _check(load().tsqr_sketch_lowp(lowp, m, n, A.data_ptr(), lda, s, seed, B.data_ptr(), s,
                                   work.data_ptr(), nbytes, _stream(stream)), "tsqr_sketch_lowp")
    return B


@_on_stream
def apply_rinv_lowp(Y: torch.Tensor, Rinv: torch.Tensor, lowp: int = FP32, stream=None):
    """X = r(Y) r(Rinv) in the low-precision type (float32 or bfloat16 tensor, column-major)."""
    ldy = _mat(Y, "Y")
    m, n = Y.shape
    ldr = _mat(Rinv, "Rinv", n, n)
    X = colmajor(m, n, device=Y.device, dtype=torch.float32 if lowp == FP32 else torch.bfloat16)
    nbytes = int(load().tsqr_rinv_lowp_bytes(n, lowp))
    work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=Y.device)
    _check(load().tsqr_apply_rinv_lowp(lowp, m, n, Y.data_ptr(), ldy, Rinv.data_ptr(), ldr,
                                       X.data_ptr(), m, work.data_ptr(), nbytes, _stream(stream)),
           "tsqr_apply_rinv_lowp")
    return X


@_on_stream
def gram_lowp(X: torch.Tensor, lowp: int = FP32, stream=None) -> torch.Tensor:
    want = torch.float32 if lowp == FP32 else torch.bfloat16
    if X.dtype != want or X.device.type != "cuda" or X.dim() != 2:
        raise ValueError(f"X must be a {want} GPU matrix")
    m, n = X.shape
    if n > 1 and m > 1 and X.stride(0) != 1:
        raise ValueError("X must be column-major")
    ldx = X.stride(1) if n > 1 else m
    W = colmajor(n, n, device=X.device)
    nbytes = int(load().tsqr_gram_workspace_bytes(m, n))
    work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=X.device)
    _check(load().tsqr_gram_lowp(lowp, m, n, X.data_ptr(), ldx, W.data_ptr(), n, work.data_ptr(),
                                 nbytes, _stream(stream)), "tsqr_gram_lowp")
    return W


@_on_stream
def rqr_cholqr(A: torch.Tensor, sketch_rows: int, seed: int, stream=None):
    """Plain form of the C ABI (stream-ordered scratch allocation, extra pass on)."""
    lda = _mat(A, "A")
    m, n = A.shape
    Q = colmajor(m, n, device=A.device)
    R = colmajor(n, n, device=A.device)
    _check(load().tsqr_rqr_cholqr(m, n, A.data_ptr(), lda, sketch_rows, seed, Q.data_ptr(),
                                  R.data_ptr(), _stream(stream)), "tsqr_rqr_cholqr")
    return Q, R


@_on_stream
def rlu_cholqr(A: torch.Tensor, sketch_rows: int, seed: int, stream=None):
    lda = _mat(A, "A")
    m, n = A.shape
    Q = colmajor(m, n, device=A.device)
    R = colmajor(n, n, device=A.device)
    _check(load().tsqr_rlu_cholqr(m, n, A.data_ptr(), lda, sketch_rows, seed, Q.data_ptr(),
                                  R.data_ptr(), _stream(stream)), "tsqr_rlu_cholqr")
    return Q, R


# ------------------------------------------------------------------------- steps ----
@_on_stream
def sketch(A: torch.Tensor, s: int, seed: int, stream=None) -> torch.Tensor:
    lda = _mat(A, "A")
    m, n = A.shape
    B = colmajor(s, n, device=A.device)
    nbytes = int(load().tsqr_sketch_workspace_bytes(m, n, s))
    work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=A.device)
    _check(load().tsqr_sketch(m, n, A.data_ptr(), lda, s, seed, B.data_ptr(), s,
                              work.data_ptr(), nbytes, _stream(stream)), "tsqr_sketch")
    return B


@_on_stream
def sketch_rows(A: torch.Tensor, s: int, seed: int, stream=None) -> torch.Tensor:
    """B = A(rows, :), the row-extraction sketch (s x n)."""
    lda = _mat(A, "A")
    m, n = A.shape
    B = colmajor(s, n, device=A.device)
    _check(load().tsqr_sketch_rows(m, n, A.data_ptr(), lda, s, seed, B.data_ptr(), s,
                                   _stream(stream)), "tsqr_sketch_rows")
    return B


@_on_stream
def sketch_factor(B: torch.Tensor, variant: int = RQR, stream=None):
    ldb = _mat(B, "B")
    s, n = B.shape
    R0 = colmajor(n, n, device=B.device)
    info = torch.zeros(1, dtype=torch.int32, device=B.device)
    nbytes = int(load().tsqr_sketch_factor_workspace_bytes(s, n))
    work = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=B.device)
    _check(load().tsqr_sketch_factor(variant, s, n, B.data_ptr(), ldb, R0.data_ptr(), n,
                                     info.data_ptr(), work.data_ptr(), nbytes,
                                     _stream(stream)), "tsqr_sketch_factor")
    return R0, info


@_on_stream
def trsm(Y: torch.Tensor, T: torch.Tensor, X: torch.Tensor | None = None, stream=None):
    ldy = _mat(Y, "Y")
    m, n = Y.shape
    ldt = _mat(T, "T", n, n)
    if X is None:
        X = colmajor(m, n, device=Y.device)
    ldx = _mat(X, "X", m, n)
    nbytes = int(load().tsqr_trsm_workspace_bytes(n))
    work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=Y.device)
    _check(load().tsqr_trsm(m, n, Y.data_ptr(), ldy, T.data_ptr(), ldt, X.data_ptr(), ldx,
                            work.data_ptr(), nbytes, _stream(stream)), "tsqr_trsm")
    return X


@_on_stream
def gram(X: torch.Tensor, stream=None) -> torch.Tensor:
    ldx = _mat(X, "X")
    m, n = X.shape
    W = colmajor(n, n, device=X.device)
    nbytes = int(load().tsqr_gram_workspace_bytes(m, n))
    work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=X.device)
    _check(load().tsqr_gram(m, n, X.data_ptr(), ldx, W.data_ptr(), n, work.data_ptr(), nbytes,
                            _stream(stream)), "tsqr_gram")
    return W


@_on_stream
def potrf(W: torch.Tensor, stage: int = 2, stream=None):
    ldw = _mat(W, "W")
    n = W.shape[0]
    R = colmajor(n, n, device=W.device)
    info = torch.zeros(1, dtype=torch.int32, device=W.device)
    _check(load().tsqr_potrf(n, W.data_ptr(), ldw, R.data_ptr(), n, stage, info.data_ptr(),
                             None, 0, _stream(stream)), "tsqr_potrf")
    return R, info


@_on_stream
def trmm_upper(A: torch.Tensor, B: torch.Tensor, stream=None) -> torch.Tensor:
    lda = _mat(A, "A")
    n = A.shape[0]
    ldb = _mat(B, "B", n, n)
    C = colmajor(n, n, device=A.device)
    _check(load().tsqr_trmm_upper(n, A.data_ptr(), lda, B.data_ptr(), ldb, C.data_ptr(), n,
                                  _stream(stream)), "tsqr_trmm_upper")
    return C


@_on_stream
def philox4x32_10(ctr: torch.Tensor, seed: int, stream=None) -> torch.Tensor:
    """ctr: (count, 4) int32 device tensor holding the counter words (bit patterns)."""
    if ctr.dtype != torch.int32 or ctr.device.type != "cuda" or ctr.dim() != 2 or ctr.shape[1] != 4:
        raise ValueError("ctr must be a (count, 4) int32 GPU tensor")
    ctr = ctr.contiguous()
    out = torch.empty_like(ctr)
    _check(load().tsqr_philox4x32_10(ctr.shape[0], ctr.data_ptr(), seed, out.data_ptr(),
                                     _stream(stream)), "tsqr_philox4x32_10")
    return out


@_on_stream
def sketch_normals(seed: int, i0: int, ni: int, j0: int, nj: int, device="cuda",
                   stream=None) -> torch.Tensor:
    Z = colmajor(ni, nj, device=device)
    _check(load().tsqr_sketch_normals(seed, i0, ni, j0, nj, Z.data_ptr(), max(ni, 1),
                                      _stream(stream)), "tsqr_sketch_normals")
    return Z


# ------------------------------------------------------------------------------ batched ----
class _Problem(ctypes.Structure):
    """Mirror of tsqr_problem (include/tsqr.h)."""
    _fields_ = [("m", _i64), ("n", _i64), ("lda", _i64), ("s", _i64), ("seed", _u64),
                ("A", _vp), ("Q", _vp), ("ldq", _i64), ("R", _vp), ("ldr", _i64)]


class BatchTuning(ctypes.Structure):
    """Mirror of tsqr_batch_tuning (include/tsqr.h)."""
    _fields_ = [("sketch_rows", _i64), ("gram_rows", _i64), ("trsm_tiles", _int)]

    def as_dict(self):
        return {"sketch_rows": self.sketch_rows, "gram_rows": self.gram_rows,
                "trsm_tiles": self.trsm_tiles}


class Batch:
    """A planned batch of independent factorizations (tsqr_batched_create).

    As: list of column-major FP64 device matrices; sketch_rows, seeds: per problem (ints or
    lists).  Q (and R unless want_r is False) are allocated here and kept alive with the
    plan, which refers to them.  run() enqueues the whole batch (kernel launches only, so it
    may be captured into a HIP graph); info is a (count,) int32 device tensor."""

    def __init__(self, As, sketch_rows, seeds, variant: int = RQR, want_r: bool = True,
                 tuning: "BatchTuning | None" = None, precision: int = 0):
        """precision: 0 (FP64 throughout), FP32 or BF16 (the sketch on that type's matrix
        cores: normals in that type, A as its FP32 rounding; every later step FP64)."""
        count = len(As)
        if count < 1:
            raise ValueError("empty batch")
        s_list = list(sketch_rows) if hasattr(sketch_rows, "__len__") else [sketch_rows] * count
        seed_list = list(seeds) if hasattr(seeds, "__len__") else [seeds] * count
        dev = As[0].device
        self.A, self.Q, self.R = list(As), [], []
        probs = (_Problem * count)()
        for i, A in enumerate(self.A):
            lda = _mat(A, f"A[{i}]")
            m, n = A.shape
            Q = colmajor(m, n, device=dev)
            R = colmajor(n, n, device=dev) if want_r else None
            self.Q.append(Q)
            self.R.append(R)
            probs[i] = _Problem(m, n, lda, s_list[i], seed_list[i], A.data_ptr(), Q.data_ptr(), m,
                                R.data_ptr() if R is not None else None, n)
        nbytes = int(load().tsqr_batched_workspace_bytes(count, ctypes.cast(probs, _vp)))
        if nbytes == 0:
            raise ValueError("invalid problem in the batch")
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.info = torch.zeros(count, dtype=torch.int32, device=dev)
        self._probs, self._variant, self._nbytes = probs, variant, nbytes
        self._precision = precision
        plan = _vp()
        _check(load().tsqr_batched_create(variant, precision, count, ctypes.cast(probs, _vp),
                                          self.work.data_ptr(), nbytes, self.info.data_ptr(),
                                          ctypes.byref(tuning) if tuning is not None else None,
                                          ctypes.byref(plan)), "tsqr_batched_create")
        self._plan = plan
        self.count = count

    def autotune(self, stream=None, persistent: bool = False):
        """Measure candidate blockings on this batch, for the phase-by-phase schedule or the
        persistent launch; returns (BatchTuning, ms per run).  Re-plans this batch with the
        winner."""
        best, ms = BatchTuning(), ctypes.c_double(0.0)
        name = "tsqr_batched_autotune_persistent" if persistent else "tsqr_batched_autotune"
        _check(getattr(load(), name)(self._variant, self._precision, self.count,
                                     ctypes.cast(self._probs, _vp), self.work.data_ptr(),
                                     self._nbytes, self.info.data_ptr(), _stream(stream),
                                     ctypes.byref(best), ctypes.byref(ms)), name)
        plan = _vp()
        _check(load().tsqr_batched_create(self._variant, self._precision, self.count,
                                          ctypes.cast(self._probs, _vp), self.work.data_ptr(),
                                          self._nbytes, self.info.data_ptr(), ctypes.byref(best),
                                          ctypes.byref(plan)), "tsqr_batched_create")
        load().tsqr_batched_destroy(self._plan)
        self._plan = plan
        return best, ms.value

    def run(self, stream=None, persistent: bool = False):
        """Enqueue the batch: one launch per phase and width class, or (persistent=True)
        one persistent kernel after a counter-clearing kernel."""
        if persistent:
            _check(load().tsqr_batched_run_persistent(self._plan, _stream(stream)),
                   "tsqr_batched_run_persistent")
        else:
            _check(load().tsqr_batched_run(self._plan, _stream(stream)), "tsqr_batched_run")

    def run_persistent_timed(self, stats: torch.Tensor, stream=None):
        """The persistent run with its scheduler time accumulated into `stats` (18 int64:
        per task kind, ticks of 10 ns waiting, in the task, and finishing the step)."""
        if stats.dtype != torch.int64 or stats.numel() < 18 or not stats.is_contiguous():
            raise ValueError("stats must be a contiguous int64 tensor of 18 entries")
        _check(load().tsqr_batched_run_persistent_timed(self._plan, stats.data_ptr(),
                                                        _stream(stream)),
               "tsqr_batched_run_persistent_timed")

    @property
    def launches(self) -> int:
        return int(load().tsqr_batched_launches(self._plan))

    @property
    def tasks(self) -> int:
        """Tasks of the persistent schedule."""
        return int(load().tsqr_batched_tasks(self._plan))

    def __del__(self):
        plan = getattr(self, "_plan", None)
        if plan is not None and plan.value is not None and _lib is not None:
            _lib.tsqr_batched_destroy(plan)
            self._plan = None
