"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function include/bf.h declares, and argument validation that
happens before any HIP call returns the documented status codes."""
import ctypes
import os
import re

import pytest

from paper_1412_4907_amd import bf

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "bf.h")


def declared_functions():
    src = open(HDR).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(bf_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_expected_api():
    names = declared_functions()
    for n in ["bf_plan_create", "bf_plan_create_ex", "bf_set_weights", "bf_run",
              "bf_plan_destroy", "bf_batch_create", "bf_batch_run", "bf_batch_destroy"]:
        assert n in names
    assert sorted(bf.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    L = bf.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


def test_strerror_and_version():
    assert bf.strerror(0) == "success"
    assert bf.strerror(bf.ERR_STATE).startswith("invalid state")
    assert bf.strerror(12345) == "unknown status"
    assert "gfx950" in bf.version()


def test_validation_before_any_device_call():
    L = bf.lib()
    h = ctypes.c_void_p()
    # bad sizes / precision / flags are rejected before the HIP runtime is touched
    assert L.bf_plan_create_ex(ctypes.byref(h), 0, 1, 1, 16, 1, 0, 0) == bf.ERR_INVALID_ARG
    assert L.bf_plan_create_ex(ctypes.byref(h), 4, 1, 1, 10, 3, 0, 0) == bf.ERR_INVALID_ARG
    assert L.bf_plan_create_ex(ctypes.byref(h), 4, 1, 1, 16, 1, 7, 0) == bf.ERR_INVALID_ARG
    assert L.bf_plan_create_ex(ctypes.byref(h), 4, 1, 1, 16, 1, 0, 8) == bf.ERR_INVALID_ARG
    # complex beam output: integration 1 only, never accumulating
    assert L.bf_plan_create_ex(ctypes.byref(h), 8, 1, 1, 16, 2, 0, bf.OUTPUT_COMPLEX) == \
        bf.ERR_INVALID_ARG
    assert L.bf_plan_create_ex(ctypes.byref(h), 8, 1, 1, 16, 1, 0,
                               bf.OUTPUT_COMPLEX | bf.ACCUMULATE) == bf.ERR_INVALID_ARG
    assert L.bf_plan_set_output_scale(None, 1.0) == bf.ERR_INVALID_ARG
    assert L.bf_set_weights_async(None, None, None, None, None) == bf.ERR_INVALID_ARG
    assert L.bf_plan_set_antenna_mask(None, None) == bf.ERR_INVALID_ARG
    assert L.bf_beam_pattern(None, None, None, None, 1, None, None) == bf.ERR_INVALID_ARG
    # 4-bit rows are read 8 antennas at a time
    assert L.bf_plan_create_ex(ctypes.byref(h), 12, 1, 1, 16, 1, 0, bf.INPUT_4BIT) == \
        bf.ERR_UNSUPPORTED
    assert L.bf_plan_create_ex(None, 4, 1, 1, 16, 1, 0, 0) == bf.ERR_INVALID_ARG
    assert L.bf_run(None, None, None, None) == bf.ERR_INVALID_ARG
    assert L.bf_set_weights(None, None, None, None, None) == bf.ERR_INVALID_ARG
    assert L.bf_plan_info(None, None) == bf.ERR_INVALID_ARG
    assert L.bf_plan_destroy(None) == bf.OK
    assert L.bf_batch_destroy(None) == bf.OK
    assert L.bf_batch_create(None, None, 1) == bf.ERR_INVALID_ARG
    # table batch: sizes, precision and 16-byte rows are checked first
    assert L.bf_table_create(None, 32, 16, 1, 0) == bf.ERR_INVALID_ARG
    assert L.bf_table_create(ctypes.byref(h), 0, 16, 1, 0) == bf.ERR_INVALID_ARG
    assert L.bf_table_create(ctypes.byref(h), 32, 0, 1, 0) == bf.ERR_INVALID_ARG
    assert L.bf_table_create(ctypes.byref(h), 32, 16, 5, 0) == bf.ERR_INVALID_ARG
    assert L.bf_table_create(ctypes.byref(h), 32, 16, 1, bf.ACCUMULATE) == bf.ERR_INVALID_ARG
    assert L.bf_table_create(ctypes.byref(h), 33, 16, 1, 0) == bf.ERR_UNSUPPORTED
    assert L.bf_table_set(None, None, None, None, 0, None) == bf.ERR_INVALID_ARG
    assert L.bf_table_run(None, None) == bf.ERR_INVALID_ARG
    assert L.bf_table_destroy(None) == bf.OK


def test_no_cpu_fallback_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(bf, "_lib", None)
    monkeypatch.setattr(bf, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        bf.lib()
