"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package holds no arithmetic of the factorization method itself: it only builds the
test matrices of the paper's experimental setup (Section 4.1) and the workload
descriptions.  Both the CPU oracle and the GPU library receive its outputs as inputs.
"""
from .matrices import (  # noqa: F401
    WORKLOADS,
    Workload,
    batched_problems,
    colmajor_padded,
    sigma_logspaced,
    gen_matrix,
    gen_ternary,
)
