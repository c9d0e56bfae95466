"""The assembly scan for vector writes placed before an exec restore at a
join (host-only, on short excerpts of gfx950 assembly)."""
from helpers.asm_check import scan

BAD = """
_ZN3qcl12_GLOBAL__N_119propagate_nN_kernelILi2E:
	s_and_saveexec_b64 s[0:1], s[56:57]
	s_xor_b64 s[0:1], exec, s[0:1]
	v_mul_f64 v[156:157], v[38:39], v[28:29]
	s_andn2_saveexec_b64 s[0:1], s[0:1]
	s_cbranch_execz .LBB18_286
	v_mul_f64 v[156:157], v[156:157], v[28:29]
.LBB18_286:                             ;   in Loop: Header=BB18_270 Depth=2
	v_accvgpr_write_b32 a84, v156
	v_accvgpr_write_b32 a85, v157
	s_mov_b32 s36, s68
	s_or_b64 exec, exec, s[0:1]
	v_mov_b32_e32 v82, v43
"""

GOOD = """
_ZN3qcl12_GLOBAL__N_119propagate_nN_kernelILi2E:
	s_and_saveexec_b64 s[0:1], s[56:57]
	s_cbranch_execz .LBB1_2
	v_mul_f64 v[156:157], v[38:39], v[28:29]
.LBB1_2:
	s_or_b64 exec, exec, s[0:1]
	v_accvgpr_write_b32 a84, v156
	v_accvgpr_write_b32 a85, v157
.LBB1_3:
	v_cmp_lt_f32_e32 vcc, 0, v1
	s_and_saveexec_b64 s[2:3], vcc
	v_mov_b32_e32 v2, 1
	s_or_b64 exec, exec, s[2:3]
"""


def test_scan_flags_copy_before_restore():
    found = scan(BAD)
    assert list(found) == ["_ZN3qcl12_GLOBAL__N_119propagate_nN_kernelILi2E"]
    (label, writes), = found["_ZN3qcl12_GLOBAL__N_119propagate_nN_kernelILi2E"]
    assert label == ".LBB18_286" and writes[0] == "v_accvgpr_write_b32 a84, v156"


def test_scan_accepts_restore_first_and_other_functions():
    assert scan(GOOD) == {}
    assert scan(BAD.replace("propagate_nN_kernel", "sym_index")) == {}  # not a kernel


# an out-of-line branch arm (the shape of the N = 5, 7 candidate factors):
# entered by execnz after the saveexec, or by falling through saveexec +
# execz, always with the arm's exec mask; its restore reads the same pair
ARM = """
_ZN3qcl12_GLOBAL__N_119propagate_nN_kernelILi7E:
	v_mov_b32_e32 v35, 0
	s_and_saveexec_b64 s[2:3], s[0:1]
	s_cbranch_execnz .LBB27_162
.LBB27_149:
	s_or_b64 exec, exec, s[2:3]
	s_branch .LBB27_170
.LBB27_161:
	v_mul_f32_e32 v58, s36, v58
	s_or_b64 exec, exec, s[4:5]
	s_and_saveexec_b64 s[2:3], s[0:1]
	s_cbranch_execz .LBB27_149
.LBB27_162:
	v_fma_f32 v35, v54, v60, 0
	v_mul_f32_e32 v35, s36, v35
	s_or_b64 exec, exec, s[2:3]
.LBB27_170:
	s_endpgm
"""


def test_scan_leaves_out_of_line_arms():
    assert scan(ARM) == {}
    # the same block also reached from an arm's last instruction is a join
    joined = ARM.replace("\ts_and_saveexec_b64 s[2:3], s[0:1]\n\ts_cbranch_execz .LBB27_149\n.LBB27_162:",
                         "\ts_and_saveexec_b64 s[2:3], s[0:1]\n\tv_mov_b32_e32 v1, 0\n.LBB27_162:")
    assert list(scan(joined)) == ["_ZN3qcl12_GLOBAL__N_119propagate_nN_kernelILi7E"]
    # or entered by a jump taken when no lane is active
    skipped = ARM.replace("s_cbranch_execnz .LBB27_162", "s_cbranch_execz .LBB27_162")
    assert list(scan(skipped)) == ["_ZN3qcl12_GLOBAL__N_119propagate_nN_kernelILi7E"]
