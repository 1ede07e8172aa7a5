"""Test matrices A = U diag(sigma) V^T with a prescribed condition number.

Recipe (paper Section 4.1, with U taken as a thin orthonormal factor):
  * G_U ~ N(0,1)^{m x n} and G_V ~ N(0,1)^{n x n} from one NumPy PCG64 stream seeded by
    ``seed`` (G_U drawn first, column-major order of draws is NumPy's row-major fill);
  * U = Q factor of G_U, V = Q factor of G_V (LAPACK Householder via NumPy);
  * sigma_k = kappa^{-k/(n-1)}, k = 0..n-1 (log-spaced from 1 down to 1/kappa), so that
    ||A||_2 = 1 and cond_2(A) = kappa up to rounding;
  * A = (U * sigma) V^T in FP64, returned column-major.
The paper builds U from a full SVD of a random m x m matrix; the thin Q factor of an
m x n Gaussian has the same (Haar) distribution on its n columns.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def sigma_logspaced(n: int, kappa: float) -> np.ndarray:
    if n == 1:
        return np.ones(1)
    k = np.arange(n, dtype=np.float64)
    return np.power(float(kappa), -k / (n - 1))


def gen_matrix(m: int, n: int, kappa: float, seed: int, dtype=np.float64) -> np.ndarray:
    """Column-major m x n FP64 matrix with singular values log-spaced in [1/kappa, 1]."""
    if m < n:
        raise ValueError("gen_matrix needs m >= n")
    rng = np.random.Generator(np.random.PCG64(seed))
    GU = rng.standard_normal((m, n))
    GV = rng.standard_normal((n, n))
    U, _ = np.linalg.qr(GU)
    del GU
    V, _ = np.linalg.qr(GV)
    sig = sigma_logspaced(n, kappa)
    U *= sig[None, :]
    A = U @ V.T
    del U
    return np.asfortranarray(A, dtype=dtype)


def gen_ternary(m: int, n: int, seed: int) -> np.ndarray:
    """Column-major m x n FP64 matrix with independent entries drawn uniformly from
    {-1, 0, 1} (many equal magnitudes: ties in a pivot search)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asfortranarray(rng.integers(-1, 2, (m, n)).astype(np.float64))


def colmajor_padded(A: np.ndarray, lda: int) -> np.ndarray:
    """Copy of A inside a column-major buffer with leading dimension ``lda`` (>= m).

    Returns the full lda x n buffer; ``buf[:m]`` is A.  Padding rows hold NaN so that a
    kernel that reads past row m is caught by the results.
    """
    m, n = A.shape
    buf = np.full((lda, n), np.nan, dtype=A.dtype, order="F")
    buf[:m] = A
    return buf


@dataclass(frozen=True)
class Workload:
    name: str
    m: int
    n: int
    s: int
    kappas: tuple
    gen_seeds: tuple
    sketch_seed: int
    extra_pass: bool
    variants: tuple = ("rqr",)
    precisions: tuple = ("fp64",)
    note: str = ""


# The five workload configurations of the benchmark specification.  Seeds are fixed so
# that every test, the smoke check and the benchmark see the same matrices.
WORKLOADS = {
    "small": Workload("small", 4096, 32, 64, (1e10,), (211101,), 11101, True,
                      note="rQR + extra pass, FP64, m=4096 n=32 s=64 kappa=1e10"),
    "tall128": Workload("tall128", 1 << 20, 128, 256, (1e14,), (211102,), 11102, True,
                        variants=("rqr", "rlu"),
                        note="rQR and rLU + extra pass, FP64, m=2^20 n=128 s=256 kappa=1e14"),
    "wide1024": Workload("wide1024", 1 << 18, 1024, 2048, (1e12,), (211103,), 11103, False,
                         note="rQR without extra pass, FP64, m=2^18 n=1024 s=2048 kappa=1e12"),
    "mixed256": Workload("mixed256", 1 << 20, 256, 512, (1e4, 1e8, 1e12),
                         (2111040, 2111041, 2111042), 11104, True,
                         precisions=("fp64", "fp32", "bf16"),
                         note="low-precision sketch/apply/first Gram, FP64 finish"),
}


def batched_problems(count: int = 512, seed: int = 211105):
    """Descriptors of the uneven batch: m ~ U[4096, 65536], n in {16,32,64,128},
    kappa = 10^U(2,10), s = 2n; per-problem generator and sketch seeds."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        m = int(rng.integers(4096, 65536, endpoint=True))
        n = int(rng.choice([16, 32, 64, 128]))
        kappa = float(10.0 ** rng.uniform(2.0, 10.0))
        out.append({"m": m, "n": n, "s": 2 * n, "kappa": kappa,
                    "gen_seed": 211105000 + i, "sketch_seed": 11105000 + i})
    return out
