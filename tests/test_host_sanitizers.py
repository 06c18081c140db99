"""Host sanitizers (CPU only): the CPU oracle and the C ABI's host code, built
with g++ -fsanitize=address,undefined and run over drivers that exercise them.

* tests/sanitize/orc_driver.cpp includes the oracle's source and runs every
  configuration family (pool types and sizes, chi-square modes, thinning,
  rotations, mu/sigma, the exponential variate, the negative controls,
  tracing), split requests of every output type, and the refused requests and
  configurations.
* tests/sanitize/abi_driver.cpp links the library's host sources (wn_api.cpp,
  wn_tune.cpp) with stand-ins for the device launchers (abi_stubs.cpp) and runs
  every path that needs no device: validation of each configuration field and
  struct version, per-stream size arrays, NULL generators at every entry
  point, the chi-square constants, the extreme-value threshold, the statistics
  battery and the tuner's argument checks.

Any sanitizer report (memory error, leak, undefined behaviour) fails the run.
The device code is not built here (GPU sanitizers are not used).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _run(exe, env_extra=None):
    env = dict(os.environ)
    env.update({"ASAN_OPTIONS": "abort_on_error=0:halt_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    env.update(env_extra or {})
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    report = r.stdout[-2000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    for marker in ("ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:"):
        assert marker not in r.stderr, report
    return r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "orc_asan")
    subprocess.run(["g++", *SAN, "-fopenmp", "-ffp-contract=off",
                    os.path.join(ROOT, "tests", "sanitize", "orc_driver.cpp"), "-o", exe],
                   check=True, timeout=600)
    out = _run(exe, {"OMP_NUM_THREADS": "4"})
    assert "failures 0" in out


@pytest.mark.skipif(shutil.which("g++") is None or
                    not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")),
                    reason="needs g++ and the HIP headers")
def test_c_abi_host_code_under_address_and_undefined_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1005_2314_amd", "csrc")
    exe = str(tmp_path / "abi_asan")
    subprocess.run(["g++", *SAN, "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
                    "-I" + os.path.join(ROOT, "include"), "-I" + csrc,
                    os.path.join(csrc, "wn_api.cpp"), os.path.join(csrc, "wn_tune.cpp"),
                    os.path.join(ROOT, "tests", "sanitize", "abi_stubs.cpp"),
                    os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp"),
                    f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib", "-o", exe],
                   check=True, timeout=600)
    # the HIP runtime keeps allocations of its own until exit: leaks are not
    # this code's; the driver's own allocations are RAII and its generators
    # are never created without a device
    out = _run(exe, {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
                     "HIP_VISIBLE_DEVICES": ""})
    assert "failures 0" in out
