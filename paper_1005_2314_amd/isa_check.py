"""Checks of the library's device assembly (run by the CPU tests).

1. Guard against a gfx950 code-generation fault seen with this library.

A wave-uniform 64-bit unsigned compare feeding a select was emitted as a VALU
compare into VCC followed by s_cselect, which reads SCC; SCC then held the
side effect of an exec-mask restore.  The kernels avoid the construct
(take_of() in wn_device.hpp); this check reads the device assembly the build
keeps and reports any s_cselect/s_cmov whose SCC can only come from an
exec-mask operation while a VALU compare into VCC sits in between.

2. The generator kernels must have no static LDS: the pool engine addresses
its LDS buffers as constants from local address 0.

3. No scalar sign extension of a 32-bit value to 64 bits in the generator
kernels.  Their counts and output offsets are unsigned; a wave-uniform 64-bit
offset rebuilt from two 32-bit words must zero-extend the low word (a
sign-extended low word with bit 31 set fills the high word with ones, and the
store goes far outside the output).
"""
import os
import re

from . import build as _build

_SCC_WRITER = re.compile(
    r"^\s+(s_cmp|s_bitcmp|s_and_|s_or_|s_xor_|s_andn2_|s_orn2_|s_nand_|s_nor_|s_xnor_|s_not_|"
    r"s_add_|s_sub_|s_addc_|s_subb_|s_lshl|s_lshr|s_ashr|s_bfe_|s_bcnt|s_min_|s_max_|s_abs_|"
    r"s_absdiff)")
_EXEC_OP = re.compile(r"^\s+s_\w+\s+(exec\b|s\[\d+:\d+\],\s*exec|exec,)")
_SCC_READER = re.compile(r"^\s+(s_cselect|s_cmov)")
_VCMP_VCC = re.compile(r"^\s+v_cmp\w*_e32\s+vcc")
_LABEL = re.compile(r"^(\.LBB|; %bb|_Z\S*:)")


def device_asm_texts():
    """Device assembly of every HIP source, as kept by the last build (built
    again first when stale or missing)."""
    files = _build.device_asm_files()
    if _build.is_stale() or not all(os.path.exists(f) for f in files):
        _build.build()
    return {os.path.basename(f): open(f).read() for f in files}


def stale_scc_selects(asm: str):
    """(kernel, line) of every select that may read a stale SCC."""
    found = []
    kernel = None
    last_writer = None
    vcmp_since = False
    for i, line in enumerate(asm.split("\n")):
        m = re.match(r"^(_Z\S*):", line)
        if m:
            kernel = m.group(1)
        if _LABEL.match(line):
            last_writer, vcmp_since = None, False
            continue
        if _SCC_READER.match(line) and vcmp_since and (
                last_writer is None or _EXEC_OP.match(last_writer)):
            found.append((kernel, i + 1))
        if _SCC_WRITER.match(line):
            last_writer, vcmp_since = line, False
        elif _VCMP_VCC.match(line):
            vcmp_since = True
    return found


_KERNEL = re.compile(r"^\s+\.amdhsa_kernel\s+(\S+)")
_STATIC_LDS = re.compile(r"^\s+\.amdhsa_group_segment_fixed_size\s+(\d+)")


def static_lds_of_engine_kernels(asm: str):
    """(kernel, bytes) for every generator kernel that declares static LDS; the
    pool engine addresses LDS from local address 0, which holds only when a
    kernel's LDS is all dynamic."""
    found = []
    kernel = None
    for line in asm.split("\n"):
        m = _KERNEL.match(line)
        if m:
            kernel = m.group(1)
            continue
        m = _STATIC_LDS.match(line)
        if m and kernel and any(k in kernel for k in ("k_fill", "k_seed")) and int(m.group(1)):
            found.append((kernel, int(m.group(1))))
    return found


_SEXT32 = re.compile(r"^\s+s_bfe_i64\s+s\[\d+:\d+\],\s*s\[\d+:\d+\],\s*0x200000\b")


def scalar_sign_extensions(asm: str):
    """(kernel, line) of every scalar 32-to-64-bit sign extension in a
    generator kernel."""
    found = []
    kernel = None
    for i, line in enumerate(asm.split("\n")):
        m = re.match(r"^(_Z\S*):", line)
        if m:
            kernel = m.group(1)
        if kernel and any(k in kernel for k in ("k_fill", "k_seed")) and _SEXT32.match(line):
            found.append((kernel, i + 1))
    return found


def check_library_sources():
    bad = []
    for name, asm in device_asm_texts().items():
        bad += [(name, k, ln) for k, ln in stale_scc_selects(asm)]
        bad += [(name, k, f"static LDS {b}") for k, b in static_lds_of_engine_kernels(asm)]
        bad += [(name, k, f"sign extension at {ln}") for k, ln in scalar_sign_extensions(asm)]
    return bad
