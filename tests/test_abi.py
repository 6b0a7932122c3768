"""The C-ABI libraries load, export every declared symbol and validate arguments (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2403_06218_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cqr_\w+)\s*\(", text)))


@pytest.mark.parametrize("header,path,sigs", [
    ("cqr.h", _native.LIB_PATH, _native.CQR_SIGNATURES),
    ("cqr_synth.h", _native.SYNTH_PATH, _native.SYNTH_SIGNATURES),
])
def test_every_declared_symbol_is_exported_and_bound(header, path, sigs):
    names = _declared(header)
    assert names, header
    lib = ctypes.CDLL(path)
    for n in names:
        assert hasattr(lib, n), "%s declared in %s but not exported" % (n, header)
    assert sorted(sigs) == names, "binding and header disagree"


def test_argument_validation_returns_lapack_style_codes():
    lib = _native.lib()
    nb = ctypes.c_size_t(0)
    assert lib.cqr_workspace_size(-1, 0, 1, ctypes.byref(nb)) == -1
    assert lib.cqr_workspace_size(4, 5, 1, ctypes.byref(nb)) == -2
    assert lib.cqr_workspace_size(4, 4, 0, ctypes.byref(nb)) == -3
    assert lib.cqr_workspace_size(400, 400, 129, ctypes.byref(nb)) == -100
    assert lib.cqr_workspace_size(1000, 500, 64, ctypes.byref(nb)) == 0 and nb.value > 1000 * 64 * 8
    flags = (ctypes.c_int32 * 4)()
    info = ctypes.c_int32(0)
    v = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation first
    assert lib.cqr_factor(-1, 1, 1, v, 1, v, 1, v, 1 << 30, ctypes.byref(info), flags, None) == -1
    assert lib.cqr_factor(3, 4, 1, v, 3, v, 4, v, 1 << 30, ctypes.byref(info), flags, None) == -2
    assert lib.cqr_factor(4, 4, 0, v, 4, v, 4, v, 1 << 30, ctypes.byref(info), flags, None) == -3
    assert lib.cqr_factor(4, 4, 2, None, 4, v, 4, v, 1 << 30, ctypes.byref(info), flags, None) == -4
    assert lib.cqr_factor(4, 4, 2, v, 3, v, 4, v, 1 << 30, ctypes.byref(info), flags, None) == -5
    assert lib.cqr_factor(4, 4, 2, v, 4, None, 4, v, 1 << 30, ctypes.byref(info), flags, None) == -6
    assert lib.cqr_factor(4, 4, 2, v, 4, v, 3, v, 1 << 30, ctypes.byref(info), flags, None) == -7
    assert lib.cqr_factor(4, 4, 2, v, 4, v, 4, None, 0, ctypes.byref(info), flags, None) == -101
    assert lib.cqr_factor(4, 4, 2, v, 4, v, 4, v, 16, ctypes.byref(info), flags, None) == -101
    assert lib.cqr_factor(4, 4, 200, v, 4, v, 4, v, 1 << 30, ctypes.byref(info), flags, None) == -100
    assert lib.cqr_orth_against(10, 4, 7, v, 10, v, 10, v, 7, v, 4, v, 1 << 30, ctypes.byref(info), None) == -3
    assert lib.cqr_orth_against(10, 4, 3, v, 10, v, 9, v, 3, v, 4, v, 1 << 30, ctypes.byref(info), None) == -7
    assert lib.cqr_solve(-1, v, 1, v, 1, v, v, 8, None) == -1
    assert lib.cqr_solve(4, v, 3, v, 4, v, v, 64, None) == -3
    assert lib.cqr_solve(4, v, 4, v, 4, v, v, 8, None) == -101
    assert b"invalid argument" in lib.cqr_status_string(-3)
    assert b"workspace" in lib.cqr_status_string(-101)
    syn = _native.synth_lib()
    assert syn.cqr_synth_uniform(-1, 1, v, 1, 0, -1.0, 1.0, None) == -1
    assert syn.cqr_synth_uniform(4, 4, v, 3, 0, -1.0, 1.0, None) == -4


def test_profiler_role_names():
    import paper_2403_06218_amd as cqr
    names = cqr.prof_names()
    assert "update" in names and "proj" in names and "chol" in names
    assert cqr.prof_query("update")["launches"] == 0
