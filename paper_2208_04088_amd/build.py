"""Builds libslbm.so (HIP, gfx950) next to this file.

    python -m paper_2208_04088_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libslbm.so")
SOURCES = [os.path.join(HERE, "csrc", "slbm.hip")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # packed fp32 instructions stay off (the compiler would otherwise form them)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no fused multiply-add contraction: every launch shape and code path
    # rounds the same expressions the same way, so results are bit-identical
    # whatever the strip width or rows per tile
    "-ffp-contract=off",
    "-Wall", "-Wno-unused-result",
    "-pthread",          # slbm_create checks large geometries on several host threads
]


def kernel_fingerprint(source="step_kernel.h"):
    """SHA-256 (16 hex digits) of a kernel source (the two-dimensional step
    kernels by default, step3_kernel.h for the three-dimensional ones) and the
    build flags: hardware-counter readings are only valid for the kernel they
    were taken on (its launch shape is recorded beside them)."""
    import hashlib
    h = hashlib.sha256()
    with open(os.path.join(HERE, "csrc", source), "rb") as fh:
        h.update(fh.read())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


def build(verbose=False, extra=()):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"),
           "-o", LIB + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
