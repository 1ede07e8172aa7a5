"""The FP64 sketch bound used by the GPU sketch tests resolves FP64 arithmetic: FP64
products of the same normals pass it in any summation order, while a product whose
operands or accumulation are FP32 fails it (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from inputs import gen_matrix
from sketch_bounds import fp64_sketch_tol


@pytest.mark.parametrize("m,n,s", [(5000, 16, 64), (3000, 128, 256)])
def test_fp64_bound_rejects_fp32_products(m, n, s):
    A = gen_matrix(m, n, 1e6, 300 + m)
    seed = 7 + n
    Z = oracle.sketch_normals(seed, 0, s, 0, m)
    rs = 1.0 / math.sqrt(s)
    ref = rs * (Z @ A)
    tol = fp64_sketch_tol(Z, A, s, ref)
    # FP64 in another order: row blocks summed back to front
    blocks = [Z[:, r:r + 512] @ A[r:r + 512] for r in range(0, m, 512)]
    acc = np.zeros_like(ref)
    for b in blocks[::-1]:
        acc += b
    assert np.all(np.abs(rs * acc - ref) <= tol)
    # the oracle's own FP64 sketch product passes as well
    assert np.all(np.abs(oracle.sketch_apply(A, s, seed) - ref) <= tol)
    # FP32 operands and FP32 accumulation
    b32 = (Z.astype(np.float32) @ A.astype(np.float32)).astype(np.float64) * rs
    r32 = np.abs(b32 - ref) / tol
    # FP32-rounded A with FP64 accumulation
    b_in = rs * (Z @ A.astype(np.float32).astype(np.float64))
    r_in = np.abs(b_in - ref) / tol
    print(f"max err/tol: fp32 gemm {r32.max():.3g}, fp32 inputs {r_in.max():.3g}")
    assert r32.max() > 100 and r_in.max() > 100
