"""The SrcC hazard check of the built kernels (paper_1412_4907_amd/isa_check):
its rule on small assembly fragments, and -- when a build's device assembly
is present -- every beamform kernel of that build."""
import glob
import os

import pytest

from paper_1412_4907_amd import isa_check

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _check(text):
    path = os.path.join(os.environ.get("TMPDIR", "/tmp"), "bf_isa_check_test.s")
    with open(path, "w") as f:
        f.write(text)
    return isa_check.check_files([path])


HEAD = "_Zkernel:\n"


def test_valu_write_of_srcc_too_soon_is_flagged():
    bad = _check(HEAD + """
    v_mfma_f32_16x16x32_bf16 v[50:53], v[38:41], v[140:143], v[26:29]
    s_nop 2
    v_perm_b32 v26, v153, v154, s42
    s_endpgm
""")
    (v,) = bad.values()
    assert v[0][2] == 3


def test_far_enough_in_place_and_loads_are_not_flagged():
    assert not _check(HEAD + """
    v_mfma_f32_16x16x32_f16 v[50:53], v[38:41], v[140:143], v[26:29]
    s_nop 6
    v_perm_b32 v26, v153, v154, s42
    v_mfma_f32_16x16x32_f16 v[60:63], v[38:41], v[140:143], v[60:63]
    v_add_u32_e32 v60, 1, v61
    v_mfma_f32_16x16x32_f16 v[70:73], v[38:41], v[140:143], v[74:77]
    ds_read_b128 v[74:77], v5
    v_mfma_f32_16x16x32_f16 v[80:83], v[38:41], v[140:143], 0
    v_mov_b32_e32 v80, 0
    s_endpgm
""")


def test_branch_targets_are_followed():
    bad = _check(HEAD + """
    v_mfma_f32_16x16x32_f16 v[50:53], v[38:41], v[140:143], v[26:29]
    s_cbranch_scc1 .LBB0_2
    s_nop 7
    s_endpgm
.LBB0_2:
    v_mov_b64_e32 v[26:27], v[8:9]
    s_endpgm
""")
    assert len(bad) == 1


def test_an_mfma_overwriting_srcc_ends_the_window():
    assert not _check(HEAD + """
    v_mfma_f32_16x16x32_f16 v[50:53], v[38:41], v[140:143], v[26:29]
    v_mfma_f32_16x16x32_f16 v[26:29], v[38:41], v[140:143], 0
    v_add_u32_e32 v26, 1, v26
    s_endpgm
""")


def test_built_kernels_pass():
    files = sorted(glob.glob(os.path.join(ROOT, "_build", "*-hip-amdgcn-amd-amdhsa-gfx950.s")))
    if not files:
        pytest.skip("no device assembly from a build in this tree")
    bad = {k: v for k, v in isa_check.check_files(files).items() if "beamform_" in k}
    assert not bad, list(bad)[:5]
