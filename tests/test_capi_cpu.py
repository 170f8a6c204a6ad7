"""C-ABI checks that need no GPU: the library loads, exports every function
include/gsis.h declares, and reports errors cleanly without a device."""
import ctypes
import os
import re

import pytest

from paper_2507_03975_amd import gsis

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gsis.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gsis_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_names():
    assert set(_declared()) == set(gsis.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = gsis.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_options_default():
    o = gsis.gsis_options()
    assert gsis.load().gsis_options_default(ctypes.byref(o)) == 0
    assert (o.method, o.precision, o.order, o.limiter, o.alsm, o.hot_face) == (1, 0, 2, 1, 1, 0)
    assert o.tol == 1e-6 and o.max_iter == 1000 and o.synth_max_iter == 50
    assert o.synth_rtol == 1e-4
    assert gsis.load().gsis_options_default(None) == gsis.GSIS_E_INVALID_ARG


def test_struct_layouts_match_header():
    # field order and sizes of the public structs (LP64)
    assert ctypes.sizeof(gsis.gsis_problem) == 4 + 4 + 8 + 8 + 8 + 7 * 8
    assert gsis.gsis_options.tol.offset == 24
    assert ctypes.sizeof(gsis.gsis_result) == 4 * 8 + 8 + 8


def test_no_device_reports_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    lib = gsis.load()
    h = ctypes.c_void_p()
    st = lib.gsis_ctx_create(0, ctypes.byref(h))
    assert st == gsis.GSIS_E_DEVICE
    assert "device" in gsis.gsis_last_error(None).lower()
    assert lib.gsis_ctx_create(0, None) == gsis.GSIS_E_INVALID_ARG
