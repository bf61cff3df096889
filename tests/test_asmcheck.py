"""The build's assembly check (paper_2312_05647_amd.asmcheck) on small
hand-written listings in clang's AMDGPU assembly format: a loop that holds a
barrier and masks lanes out of itself is reported; the same loop with a
uniform (scalar) exit, and a divergent loop without a barrier, are not."""
from paper_2312_05647_amd import asmcheck

DIVERGENT = """
_ZN3mjp4k_badEv:                        ; @_ZN3mjp4k_badEv
; %bb.0:
	s_branch .LBB0_2
.LBB0_1:                                ;   in Loop: Header=BB0_2 Depth=1
	s_andn2_b64 exec, exec, s[4:5]
	s_cbranch_execz .LBB0_3
.LBB0_2:                                ; =>This Loop Header: Depth=1
	s_waitcnt lgkmcnt(0)
	s_barrier
	ds_read_b32 v0, v1
	s_branch .LBB0_1
.LBB0_3:
	s_endpgm
.Lfunc_end0:
"""

UNIFORM = """
_ZN3mjp5k_goodEv:                       ; @_ZN3mjp5k_goodEv
; %bb.0:
	s_branch .LBB1_2
.LBB1_1:                                ;   in Loop: Header=BB1_2 Depth=1
	s_cmp_ge_i32 s4, s33
	s_cbranch_scc1 .LBB1_3
.LBB1_2:                                ; =>This Loop Header: Depth=1
	s_waitcnt lgkmcnt(0)
	s_barrier
	v_readfirstlane_b32 s4, v0
	s_branch .LBB1_1
.LBB1_3:
	s_endpgm
.Lfunc_end1:
"""

NO_BARRIER = """
_ZN3mjp6k_spinEv:                       ; @_ZN3mjp6k_spinEv
; %bb.0:
.LBB2_1:                                ; =>This Loop Header: Depth=1
	global_load_dword v0, v[2:3], off
	s_andn2_b64 exec, exec, s[4:5]
	s_cbranch_execnz .LBB2_1
; %bb.2:
	s_endpgm
.Lfunc_end2:
"""


def test_reports_divergent_loop_with_barrier():
    assert asmcheck.divergent_barrier_loops(DIVERGENT) == [("_ZN3mjp4k_badEv", "BB0_2")]


def test_uniform_loop_and_barrier_free_loop_pass():
    assert asmcheck.divergent_barrier_loops(UNIFORM) == []
    assert asmcheck.divergent_barrier_loops(NO_BARRIER) == []
    assert asmcheck.divergent_barrier_loops(UNIFORM + DIVERGENT) == [("_ZN3mjp4k_badEv", "BB0_2")]
