"""Host checks of the build script: every source it compiles exists, the units with
extra flags are compiled, and the scratch check reads the compiler's resource-usage
remarks (a streaming kernel with private memory fails the build, other kernels and
streaming kernels without it pass)."""
import os

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
