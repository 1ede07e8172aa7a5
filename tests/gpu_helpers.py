"""Helpers for the GPU tests: host/device transfers and blocked FP64 accuracy metrics.

The metrics on the device use torch's FP64 matrix products on 4096-row blocks and a
pairwise (tree) sum of the block results, so that their own rounding stays near
u*sqrt(4096) relative instead of u*sqrt(m); they are cross-checked against the oracle's
double-double metrics at small sizes in the tests.
"""
import numpy as np
import torch

BLOCK = 4096


def host(t: torch.Tensor) -> np.ndarray:
    return np.asfortranarray(t.detach().cpu().numpy())


def _tree_sum(parts):
    while len(parts) > 1:
        nxt = [parts[i] + parts[i + 1] for i in range(0, len(parts) - 1, 2)]
        if len(parts) % 2:
            nxt.append(parts[-1])
        parts = nxt
    return parts[0]


def gpu_orthogonality(Q: torch.Tensor) -> float:
    m, n = Q.shape
    parts = []
    for r0 in range(0, m, BLOCK):
        blk = Q[r0:r0 + BLOCK].contiguous()
        parts.append(blk.t().contiguous() @ blk)
    G = _tree_sum(parts)
    G -= torch.eye(n, dtype=G.dtype, device=G.device)
    return float(torch.linalg.matrix_norm(G).item())


def gpu_residual(A: torch.Tensor, Q: torch.Tensor, R: torch.Tensor) -> float:
    m, n = A.shape
    num, den = [], []
    Rc = R.contiguous()
    for r0 in range(0, m, BLOCK):
        a = A[r0:r0 + BLOCK]
        e = a - Q[r0:r0 + BLOCK].contiguous() @ Rc
        num.append((e * e).sum())
        den.append((a * a).sum())
    return float(torch.sqrt(_tree_sum(num)).item() / torch.sqrt(_tree_sum(den)).item())


def rel_fro(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
