"""The C-ABI library loads and exports every symbol include/smartap.h
declares; argument checks that need no device return error codes."""
import ctypes as C
import os
import re

import pytest

from paper_2609_11181_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "smartap.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(smart_[a-z_0-9]+)\s*\(", src)))


def test_exports_match_header():
    lib = L.load()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTS) == names


def test_null_arguments_fail_cleanly():
    lib = L.load()
    assert lib.smart_init(0, None) == L.EINVAL
    assert lib.smart_run(None, 0, None, None) == L.EINVAL
    fid = C.c_int()
    assert lib.smart_filter_define(None, 0, None, 0, C.byref(fid)) == L.EINVAL
    assert lib.smart_plan_create(None, None, 0, 64, 0, None, 1, None, None, 1, None, None) == L.EINVAL
    assert lib.smart_data_info(None, None, None, None, None, None) == L.EINVAL
    assert lib.smart_last_error().decode() != ""
    assert b"gfx950" in lib.smart_version()


def test_enums_match_header():
    src = open(os.path.join(ROOT, "include", "smartap.h")).read()
    for name, val in [("SMART_FILTER_TANH", L.FILTER_TANH), ("SMART_VAR_PIXEL", L.VAR_PIXEL),
                      ("SMART_PREC_BF16X3", L.PREC_BF16X3), ("SMART_NORM_RAW", L.NORM_RAW),
                      ("SMART_EUNSUPPORTED", L.EUNSUPPORTED), ("SMART_PREC_FP32_OUT64", L.PREC_FP32_OUT64),
                      ("SMART_FILTER_TABLE", L.FILTER_TABLE), ("SMART_NORM_AVERAGED", L.NORM_AVERAGED)]:
        m = re.search(rf"{name}\s*=\s*(-?\d+)", src)
        assert m and int(m.group(1)) == val, name


@pytest.mark.parametrize("name", ["smart_free_everything", "smart_magic"])
def test_no_unknown_symbols(name):
    assert not hasattr(L.load(), name)
