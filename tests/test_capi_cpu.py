"""C-ABI checks that need no GPU: the library loads, exports every function
include/gsis.h declares, and reports errors cleanly without a device."""
import ctypes
import os
import re
import subprocess

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
    assert o.synth_rtol == 0.1 and o.cfl_p == 0.0 and o.beta == 0.0
    assert gsis.load().gsis_options_default(None) == gsis.GSIS_E_INVALID_ARG


def test_struct_layouts_match_header(tmp_path):
    """Offsets and sizes of the public structs as the C compiler lays them out
    from include/gsis.h equal the binding's ctypes layouts."""
    structs = [gsis.gsis_problem, gsis.gsis_options, gsis.gsis_result]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gsis.h"', "int main(void) {"]
    for st in structs:
        n = st.__name__
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (n, n))
        for f in st._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (n, f[0], n, f[0]))
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                           str(src)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for st in structs:
        n = st.__name__
        assert int(got[n]) == ctypes.sizeof(st), n
        for f in st._fields_:
            assert int(got["%s.%s" % (n, f[0])]) == getattr(st, f[0]).offset, (n, f[0])


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
