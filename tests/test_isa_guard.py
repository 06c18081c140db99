"""The device code must not contain selects that can read a stale SCC, static
LDS in the generator kernels, or scalar sign extensions of 32-bit words into
64-bit offsets (see paper_1005_2314_amd/isa_check.py); the check
cross-compiles on the CPU."""
from paper_1005_2314_amd import isa_check


def test_checker_flags_the_known_bad_sequence():
    bad = """_Zbad:
	s_or_b64 exec, exec, s[0:1]
	v_cmp_lt_u64_e32 vcc, s[52:53], v[26:27]
	s_cselect_b32 s6, s52, 0x3ff
"""
    good = """_Zgood:
	v_cmp_lt_u64_e32 vcc, s[16:17], v[0:1]
	s_and_b64 s[0:1], vcc, exec
	s_cselect_b32 s24, s16, s38
"""
    assert isa_check.stale_scc_selects(bad) == [("_Zbad", 4)]
    assert isa_check.stale_scc_selects(good) == []


def test_library_device_code_has_no_stale_scc_select():
    assert isa_check.check_library_sources() == []


def test_static_lds_checker():
    asm = """	.amdhsa_kernel _Z6k_fillv
		.amdhsa_group_segment_fixed_size 16
	.amdhsa_kernel _Z6k_sumv
		.amdhsa_group_segment_fixed_size 64
"""
    assert isa_check.static_lds_of_engine_kernels(asm) == [("_Z6k_fillv", 16)]


def test_sign_extension_checker():
    asm = """_Z6k_fillv:
	s_mov_b32 s61, s11
	s_bfe_i64 s[8:9], s[10:11], 0x200000
	s_or_b64 s[90:91], s[8:9], s[60:61]
_Z5otherv:
	s_bfe_i64 s[8:9], s[10:11], 0x200000
"""
    assert isa_check.scalar_sign_extensions(asm) == [("_Z6k_fillv", 3)]
