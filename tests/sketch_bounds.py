"""Error bound of an FP64 sketch product B = rs (Z A), rs = 1/sqrt(s), shared by the GPU
sketch tests and the CPU test that shows the bound rejects an FP32 product.

Any FP64 summation order of the m products z_ij a_jc (the device's row blocks on the
matrix cores and the fixed-order sum of their partials, or NumPy's) is within
gamma_m sum_j |z_ij a_jc| of the exact sum, gamma_m = m u / (1 - m u) <= 1.01 m u.  Two
such sums (device and reference) differ by at most twice that; each is then scaled by rs
with one more rounding.  The bound below allows 4 m u, twice the worst case.
"""
import math

import numpy as np

U = 2.0 ** -53


def fp64_sketch_tol(Z: np.ndarray, A: np.ndarray, s: int, B_ref: np.ndarray) -> np.ndarray:
    m = A.shape[0]
    rs = 1.0 / math.sqrt(s)
    return rs * 4 * m * U * (np.abs(Z) @ np.abs(A)) + 4 * U * np.abs(B_ref)
