"""The build's check that no forward or adjoint kernel uses scratch memory,
on the compiler's kernel-resource-usage remarks (no compiler run)."""
import pytest

from paper_2601_00551_amd import build

REMARKS = """\
x.hip:367:1: remark: Function Name: _ZN3sbp9k_adjointIfLi1ELi1ELb1EEEvNS_6ArrayP [-Rpass-analysis=kernel-resource-usage]
x.hip:367:1: remark:     VGPRs: 128 [-Rpass-analysis=kernel-resource-usage]
x.hip:367:1: remark:     ScratchSize [bytes/lane]: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:367:1: remark:     SGPRs Spill: 12 [-Rpass-analysis=kernel-resource-usage]
x.hip:367:1: remark:     VGPRs Spill: 0 [-Rpass-analysis=kernel-resource-usage]
x.hip:481:1: remark: Function Name: _ZN3sbp12k_adj_reduceIfLb1EE [-Rpass-analysis=kernel-resource-usage]
x.hip:481:1: remark:     ScratchSize [bytes/lane]: 16 [-Rpass-analysis=kernel-resource-usage]
x.hip:481:1: remark:     VGPRs Spill: 3 [-Rpass-analysis=kernel-resource-usage]
"""


def test_remarks_parse():
    u = build.resource_usage(REMARKS)
    assert u["_ZN3sbp9k_adjointIfLi1ELi1ELb1EEEvNS_6ArrayP"]["VGPRs"] == 128
    assert u["_ZN3sbp9k_adjointIfLi1ELi1ELb1EEEvNS_6ArrayP"]["SGPRs Spill"] == 12
    assert u["_ZN3sbp12k_adj_reduceIfLb1EE"]["ScratchSize [bytes/lane]"] == 16


def test_scratch_in_a_physics_kernel_fails_the_build():
    # SGPR spills (to VGPR lanes) and scratch in a non-physics kernel pass
    build.check_no_scratch(build.resource_usage(REMARKS), "x.hip")
    bad = REMARKS.replace("ScratchSize [bytes/lane]: 0", "ScratchSize [bytes/lane]: 8", 1)
    with pytest.raises(RuntimeError, match="scratch"):
        build.check_no_scratch(build.resource_usage(bad), "x.hip")
    bad = REMARKS.replace("VGPRs Spill: 0", "VGPRs Spill: 1", 1)
    with pytest.raises(RuntimeError, match="k_adjoint"):
        build.check_no_scratch(build.resource_usage(bad), "x.hip")
