"""The C-ABI libraries load, export every declared symbol and validate arguments (no GPU needed)."""
import ctypes
import os
import re

import pytest
import torch

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
    assert lib.cqr_workspace_size(400, 400, 257, ctypes.byref(nb)) == -100
    assert lib.cqr_workspace_size(1000, 500, 64, ctypes.byref(nb)) == 0 and nb.value > 1000 * 64 * 8
    v = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation first
    info = flags = v
    assert lib.cqr_factor(-1, 1, 1, v, 1, v, 1, v, 1 << 30, info, flags, None) == -1
    assert lib.cqr_factor(3, 4, 1, v, 3, v, 4, v, 1 << 30, info, flags, None) == -2
    assert lib.cqr_factor(4, 4, 0, v, 4, v, 4, v, 1 << 30, info, flags, None) == -3
    assert lib.cqr_factor(4, 4, 2, None, 4, v, 4, v, 1 << 30, info, flags, None) == -4
    assert lib.cqr_factor(4, 4, 2, v, 3, v, 4, v, 1 << 30, info, flags, None) == -5
    assert lib.cqr_factor(4, 4, 2, v, 4, None, 4, v, 1 << 30, info, flags, None) == -6
    assert lib.cqr_factor(4, 4, 2, v, 4, v, 3, v, 1 << 30, info, flags, None) == -7
    assert lib.cqr_factor(4, 4, 2, v, 4, v, 4, None, 0, info, flags, None) == -101
    assert lib.cqr_factor(4, 4, 2, v, 4, v, 4, v, 16, info, flags, None) == -101
    assert lib.cqr_factor(4, 4, 300, v, 4, v, 4, v, 1 << 30, info, flags, None) == -100
    assert lib.cqr_orth_against(10, 4, 7, v, 10, v, 10, v, 7, v, 4, v, 1 << 30, info, None) == -3
    assert lib.cqr_orth_against(10, 4, 3, v, 10, v, 9, v, 3, v, 4, v, 1 << 30, info, None) == -7
    assert lib.cqr_solve(-1, v, 1, v, 1, v, v, 8, v, None) == -1
    assert lib.cqr_solve(4, v, 3, v, 4, v, v, 64, v, None) == -3
    assert lib.cqr_solve(4, v, 4, v, 4, v, v, 8, v, None) == -101
    assert lib.cqr_set_wait_limit_us(-1) == -1
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


def test_batched_validation_and_plan():
    lib = _native.lib()
    v = ctypes.c_void_p(0x1000)  # never dereferenced: every case fails validation first
    nb = ctypes.c_size_t(0)
    assert lib.cqr_batched_workspace_size(-1, ctypes.byref(nb)) == -1
    assert lib.cqr_batched_workspace_size(10000, ctypes.byref(nb)) == 0 and nb.value >= 40000
    assert lib.cqr_batched_factor_solve(0, 0, None, None, None, None, None, None, None, None, None, 0, None) == 0
    assert lib.cqr_batched_factor_solve(-1, 0, v, v, v, v, v, v, v, v, v, 1 << 20, None) == -1
    assert lib.cqr_batched_factor_solve(4, 2, v, v, v, v, v, v, v, v, v, 1 << 20, None) == -2
    assert lib.cqr_batched_factor_solve(4, 0, None, v, v, v, v, v, v, v, v, 1 << 20, None) == -3
    assert lib.cqr_batched_factor_solve(4, 0, v, v, v, None, v, v, v, v, v, 1 << 20, None) == -6
    assert lib.cqr_batched_factor_solve(4, 0, v, v, v, v, v, v, None, v, v, 1 << 20, None) == -9
    assert lib.cqr_batched_factor_solve(4, 1, v, v, v, v, v, v, v, v, v, 8, None) == -101
    from paper_2403_06218_amd import batched
    insts = batched.instances()
    assert len(insts) >= 4 and {i["dtype"] for i in insts} == {0, 1}
    assert all(i["bw"] in (16, 32) and i["nmax"] in (64, 128, 256, 512) for i in insts)
    for dt in (torch.float64, torch.float32):
        plan = batched.get_plan(dt)
        assert plan["hi"][-1] == 512 and plan["hi"] == sorted(plan["hi"])
        for h, i in zip(plan["hi"], plan["inst"]):
            assert insts[i]["nmax"] >= h and insts[i]["dtype"] == (0 if dt == torch.float64 else 1)
    f64_256 = next(i["id"] for i in insts if i["dtype"] == 0 and i["nmax"] == 256)
    f32_any = next(i["id"] for i in insts if i["dtype"] == 1)
    with pytest.raises(_native.CqrError):
        batched.set_plan(torch.float64, [512], [f64_256])       # nmax too small for the bucket
    with pytest.raises(_native.CqrError):
        batched.set_plan(torch.float64, [64, 32], [f64_256, f64_256])  # bounds not ascending
    with pytest.raises(_native.CqrError):
        batched.set_plan(torch.float64, [64], [f32_any])        # wrong element type
    old = batched.get_plan(torch.float64)
    batched.set_plan(torch.float64, [100, 256], [f64_256, f64_256])
    assert batched.get_plan(torch.float64) == {"hi": [100, 256], "inst": [f64_256, f64_256]}
    assert batched.block_width(100) == insts[f64_256]["bw"]
    batched.set_plan(torch.float64, old["hi"], old["inst"])


def test_qr_solve_rejects_sizes_above_the_plan():
    # A host-side check before any device work: above the plan's largest size
    # the kernels would skip the matrix and leave x = b.
    from paper_2403_06218_amd import batched
    top = batched.get_plan(torch.float64)["hi"][-1]
    A = torch.zeros(2, top + 1, top + 1, dtype=torch.float64)
    b = torch.zeros(2, top + 1, dtype=torch.float64)
    with pytest.raises(ValueError, match="largest size"):
        batched.qr_solve(A, b)
