"""Build ``paper_2111_11148_amd/libtsqr.so`` from the HIP sources in ``csrc/`` for gfx950.

Each translation unit (every ``.hip`` file except the parts that ``k_chain.hip`` includes)
is compiled to an object in ``_build/`` (in parallel), then linked into one shared library
exporting the C ABI of ``include/tsqr.h``.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libtsqr.so")
ARCH = os.environ.get("TSQR_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(_ROOT, "include"),
]


def _compile(src: str, obj: str, verbose: bool) -> None:
    cmd = [HIPCC, *CFLAGS, "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip() and verbose:
        print(err, flush=True)


# Sources compiled only as part of k_chain.hip (one translation unit, so that the persistent
# batched kernel can inline the device bodies of every phase).
CHAIN_PARTS = {"k_sketch.hip", "k_tall.hip", "k_small.hip", "k_lowp.hip", "k_persist.hip"}


def build(verbose: bool = False) -> str:
    srcs = sorted(s for s in glob.glob(os.path.join(_HERE, "csrc", "*.hip"))
                  if os.path.basename(s) not in CHAIN_PARTS)
    bdir = os.path.join(_ROOT, "_build", "tsqr")
    os.makedirs(bdir, exist_ok=True)
    objs = [os.path.join(bdir, os.path.basename(s)[:-4] + ".o") for s in srcs]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose), zip(srcs, objs)))
    tmp = LIB_PATH + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
