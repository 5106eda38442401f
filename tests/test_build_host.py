"""Host checks of the build script: every source it compiles exists, the units with
extra flags are compiled, the scratch check reads the compiler's resource-usage
remarks (a streaming kernel with private memory fails the build, other kernels and
streaming kernels without it pass), and no store of more than 64 bits in the wide
streaming kernel has its data registers rewritten by the next instruction."""
import os

import pytest

from paper_2411_18341_amd import build

REMARKS = """\
x.hip:9:1: remark: Function Name: _ZN3phx24rk4_stream_spinor_kernelIfLb1EEEvv [-Rpass-analysis=kernel-resource-usage]
x.hip:9:1: remark:     VGPRs: 147 [-Rpass-analysis=kernel-resource-usage]
x.hip:9:1: remark:     ScratchSize [bytes/lane]: 288 [-Rpass-analysis=kernel-resource-usage]
    9 | {
      | ^
x.hip:9:1: remark: Function Name: _ZN3phx24rk4_stream_spinor_kernelIfLb0EEEvv [-Rpass-analysis=kernel-resource-usage]
x.hip:9:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:9:1: remark: Function Name: _ZN3phx14dp_stage_kernelIfEEvv [-Rpass-analysis=kernel-resource-usage]
x.hip:9:1: remark:     ScratchSize [bytes/lane]: 64 [-Rpass-analysis=kernel-resource-usage]
"""


def test_sources_exist_and_flagged_units_are_built():
    for s in build.SOURCES:
        assert os.path.exists(os.path.join(build.CSRC, s)), s
    assert set(build.EXTRA_FLAGS) <= set(build.SOURCES)
    assert build.STREAM_SOURCES <= set(build.SOURCES)
    assert len(set(build.SOURCES)) == len(build.SOURCES)


def test_scratch_check_reads_the_remarks():
    assert build._scratch_kernels(REMARKS) == [("_ZN3phx24rk4_stream_spinor_kernelIfLb1EEEvv", 288)]
    assert build._scratch_kernels(REMARKS.replace("288", "0")) == []
    assert build._scratch_kernels("") == []


ASM = """\
_Z1kv:                                  ; @_Z1kv
; %bb.0:
\tbuffer_store_dwordx4 v[8:11], v2, s[0:3], s4 offen nt
\tv_mov_b32_e32 v10, s5
\tbuffer_store_dwordx4 v[12:15], v2, s[0:3], 0 offen nt
\ts_nop 0
\tv_mov_b32_e32 v12, s5
\tbuffer_store_dwordx2 v[16:17], v2, s[0:3], s4 offen
\tv_mov_b32_e32 v16, s5
\tglobal_store_dwordx4 v[0:1], v[20:23], off
.LBB0_1:
\tv_mov_b32_e32 v20, s5
\tbuffer_store_dwordx4 v[24:27], v2, s[0:3], s4 offen
\tv_add_f32_e32 v30, v24, v25
\tv_cmp_gt_f32_e32 vcc, v24, v26
\tv_fma_f32 v27, v1, v2, v3
\ts_endpgm
"""


def test_store_hazard_scan_on_a_listing():
    """The scan flags a 128-bit store whose data the next instruction rewrites, and
    nothing else: a wait state in between, 64-bit stores, a block boundary, reads of
    the data and compares are fine; a wider window also catches the last store."""
    found = build.store_data_hazards(ASM)
    assert [(f, st.split()[1]) for f, st, _ in found] == [("_Z1kv", "v[8:11],")]
    wider = build.store_data_hazards(ASM, min_gap=4)
    assert [st.split()[1] for _, st, _ in wider] == ["v[8:11],", "v[12:15],", "v[24:27],"]


@pytest.mark.parametrize("unit", ["rk4_stream_wide.hip", "batch.hip"])
def test_wide_kernel_stores_keep_their_data(unit):
    """Every 128-bit store of the wide streaming walk (single grid and batched) has at
    least one instruction before a VALU write to its data registers (device assembly
    of the unit, built with the library's flags)."""
    asm = build.device_asm(unit)
    assert "buffer_store_dwordx4" in asm
    assert build.store_data_hazards(asm) == []
