"""Build the CPU oracle (test infrastructure) into ``oracle/liborc.so``.

The flags matter: ``-ffp-contract=off`` and no fast-math keep every floating
point operation a single correctly rounded IEEE-754 operation, in the order the
source states it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wn_oracle.cpp")
LIB = os.path.join(HERE, "liborc.so")

FLAGS = ["-std=c++17", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
         "-fno-fast-math", "-mfpmath=sse", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    cmd = ["g++", *FLAGS, SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
