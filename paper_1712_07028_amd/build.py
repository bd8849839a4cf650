"""Build the HIP library libfsl.so (gfx950) in the package directory, and two
helpers: libfsl_checks.so (host builds of two pure functions of its kernels, for
tests) and libfsl_ceiling.so (the pull with no arithmetic, a bandwidth ceiling for
the benchmark)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfsl.so")
SOURCES = [os.path.join(CSRC, "fsl_api.hip")]
CHECKS_LIB = os.path.join(HERE, "libfsl_checks.so")
CHECKS_SOURCES = [os.path.join(CSRC, "fsl_checks.hip")]
CEILING_LIB = os.path.join(HERE, "libfsl_ceiling.so")
CEILING_SOURCES = [os.path.join(CSRC, "fsl_ceiling.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-shared", "-fPIC",
    "-munsafe-fp-atomics",
    # packed FP32 instructions stay off (plain scalar float code only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the kernels index their per-cell population arrays with constants only, so
    # they live in scalar registers; promoting them to vector values instead makes
    # every conditional update copy the whole vector (and spill)
    "-mllvm", "-disable-promote-alloca-to-vector",
    "-Wall", "-Werror=return-type",
]


def _compile(lib, sources, verbose):
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *sources]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=CSRC)
    os.replace(tmp, lib)


def build(verbose=False):
    """Compile libfsl.so and libfsl_checks.so; always recompiles."""
    _compile(LIB, SOURCES, verbose)
    _compile(CHECKS_LIB, CHECKS_SOURCES, verbose)
    _compile(CEILING_LIB, CEILING_SOURCES, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
