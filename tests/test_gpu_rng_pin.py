"""Pin of the oracle's Philox4x32-10 against rocRAND's independent implementation.

rocRAND's host-side PHILOX4_32_10 generator needs the HIP runtime, so this runs on the
GPU machine.  rocRAND keys the generator with (low, high) 32-bit halves of the seed and
walks counters (c0, c1, c2, c3) with the block index in (c0, c1) and a subsequence index
in (c2, c3); every aligned block of four words it emits must therefore be one Philox call
of the oracle with such a counter.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle

ROCRAND = "/opt/rocm/lib/librocrand.so"
PHILOX4_32_10 = 404


@pytest.mark.gpu
def test_oracle_philox4x32_matches_rocrand(gpu_available):
    if not os.path.exists(ROCRAND):
        pytest.skip("rocRAND not installed")
    lib = ctypes.CDLL(ROCRAND)
    gen = ctypes.c_void_p()
    assert lib.rocrand_create_generator_host_blocking(ctypes.byref(gen), PHILOX4_32_10) == 0
    try:
        for seed in (0, 11102, 0x123456789ABCDEF):
            assert lib.rocrand_set_seed(gen, ctypes.c_ulonglong(seed)) == 0
            out = np.zeros(1024, dtype=np.uint32)
            st = lib.rocrand_generate(gen, out.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(out.size))
            assert st == 0, f"rocrand_generate status {st}"
            key = [seed & 0xFFFFFFFF, seed >> 32]
            table = {}
            for c0 in range(512):
                for c2 in range(4):
                    w = oracle.philox4x32_10([c0, 0, c2, 0], key)
                    table[tuple(int(x) for x in w)] = (c0, c2)
            blocks = [tuple(int(x) for x in out[i:i + 4]) for i in range(0, out.size, 4)]
            found = sum(b in table for b in blocks)
            print(f"seed={seed:#x}: {found}/{len(blocks)} rocRAND blocks found among oracle blocks",
                  flush=True)
            assert found == len(blocks)
    finally:
        lib.rocrand_destroy_generator(gen)
