"""Build the gfx950 library ``libwn.so`` in-tree with hipcc.

Every HIP source is compiled for gfx950 only, with floating-point contraction
off (bit-exact IEEE operations in source order) and packed-FP32 instructions
disabled.  ``build(poison=True)`` builds the debug variant ``libwn_poison.so``
(WN_POISON_LDS=1: every LDS pool write is preceded by a NaN fill of the
buffer), which the binding loads when WN_LDS_POISON=1 is set.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwn.so")
POISON_LIB = os.path.join(HERE, "libwn_poison.so")
# one launch unit per (pool type, output type), compiled in parallel
LAUNCH_UNITS = ("wn_launch_f32_f32.hip", "wn_launch_f32_bf16.hip", "wn_launch_f32_f16.hip",
                "wn_launch_f64_f64.hip", "wn_launch_f64_f32.hip", "wn_launch_f64_bf16.hip",
                "wn_launch_f64_f16.hip")
SOURCES = [os.path.join(CSRC, f) for f in
           LAUNCH_UNITS + ("wn_stats.hip", "wn_noalloc.hip", "wn_bench.hip", "wn_api.cpp",
                             "wn_tune.cpp")]
HEADERS = [os.path.join(CSRC, f) for f in ("wn_internal.hpp", "wn_device.hpp", "wn_launch.hpp")] + [
    os.path.join(ROOT, "include", "wn.h"), os.path.join(ROOT, "include", "wn_bench.h")]
BUILD_DIR = os.path.join(ROOT, "_build")
POISON_BUILD_DIR = os.path.join(ROOT, "_build_poison")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def _compile(src: str, verbose: bool, poison: bool = False) -> str:
    """Compile one source to an object in _build/ (_build_poison/ for the debug
    variant), keeping the device assembly (*-hip-amdgcn-amd-amdhsa-gfx950.s)
    beside it for the ISA guard."""
    bdir = POISON_BUILD_DIR if poison else BUILD_DIR
    obj = os.path.join(bdir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *[f for f in FLAGS if f != "-shared"], *(["-DWN_POISON_LDS=1"] if poison else []),
           "-save-temps=obj", "-c", "-x", "hip", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=bdir)
    return obj


def build(verbose: bool = False, poison: bool = False) -> str:
    """Build libwn.so, or with poison=True the debug variant libwn_poison.so."""
    from concurrent.futures import ThreadPoolExecutor
    bdir, lib = (POISON_BUILD_DIR, POISON_LIB) if poison else (BUILD_DIR, LIB)
    os.makedirs(bdir, exist_ok=True)
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        objs = list(pool.map(lambda src: _compile(src, verbose, poison), SOURCES))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", lib + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


def device_asm_files():
    """Device assembly kept by the last build, one per HIP source."""
    out = []
    for src in SOURCES:
        if src.endswith(".hip"):
            stem = os.path.splitext(os.path.basename(src))[0]
            out.append(os.path.join(BUILD_DIR, f"{stem}-hip-amdgcn-amd-amdhsa-gfx950.s"))
    return out


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS + [__file__])


if __name__ == "__main__":
    build(verbose=True, poison="--poison" in sys.argv[1:])
    sys.exit(0)
