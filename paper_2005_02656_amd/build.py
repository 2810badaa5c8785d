"""Builds libsph.so (the HIP library behind include/sph.h) in-tree for gfx950.

    python -m paper_2005_02656_amd.build

Every call compiles every source (the build check must not trust a stale
library).  Objects go to paper_2005_02656_amd/_build/, the shared library to
paper_2005_02656_amd/libsph.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsph.so")
SOURCES = ["sph_api.hip", "sph_cells.hip", "sph_search.hip", "sph_pairs.hip",
           "sph_mixed.hip", "sph_integrate.hip", "sph_adjoint.hip", "sph_gravity.hip"]
ARCH = os.environ.get("SPH_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # the neighbour test and the keys round identically to the definition only
    # without contraction; fused multiply-adds are written explicitly (fma())
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _compile(src: str, build_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, extra_flags=(), out: str = LIB) -> str:
    """Compiles every source and links `out`; extra_flags (e.g. tuning -D
    macros) go to every compile, and their objects to a directory of their own."""
    build_dir = BUILD if not extra_flags else os.path.join(
        BUILD, "v" + str(abs(hash(tuple(extra_flags))) % 10**8))
    os.makedirs(build_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, build_dir, extra_flags), SOURCES))
    LIB_OUT = out
    tmp = LIB_OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_OUT)
    if verbose:
        print(LIB_OUT)
    return LIB_OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
