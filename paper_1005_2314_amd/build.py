"""Build the gfx950 library ``libwn.so`` in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with floating-point contraction
off (bit-exact IEEE operations in source order) and packed-FP32 instructions
disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwn.so")
SOURCES = [os.path.join(CSRC, f) for f in ("wn_kernels.hip", "wn_bench.hip", "wn_api.cpp")]
HEADERS = [os.path.join(CSRC, "wn_internal.hpp"), os.path.join(ROOT, "include", "wn.h"),
           os.path.join(ROOT, "include", "wn_bench.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def build(verbose: bool = False) -> str:
    cmd = [HIPCC, *FLAGS, "-x", "hip", *SOURCES, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
