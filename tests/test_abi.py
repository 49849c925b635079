"""C-ABI checks that need no GPU: the library loads, exports every symbol the header declares, and
rejects invalid arguments on the host before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slhjb.h")


@pytest.fixture(scope="module")
def slhjb():
    import paper_1605_04821_amd as m
    return m


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hjb_[a-z_]+)\s*\(", txt)))


def test_header_symbols_exported(slhjb):
    names = _declared()
    assert "hjb_setup" in names and "hjb_step" in names and "hjb_solve" in names and "hjb_policy_sweep" in names
    out = subprocess.run(["nm", "-D", "--defined-only", slhjb.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (hjb_[a-z_]+)\b", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(slhjb.lib(), n)
    assert sorted(slhjb.EXPORTED) == sorted(names)


def _desc(slhjb, **kw):
    d = slhjb.Desc()
    slhjb.lib().hjb_desc_default(ctypes.byref(d))
    d.dim = 2
    d.n[0] = d.n[1] = 9
    d.n[2] = 1
    d.h = 1.0 / 8
    d.K, d.P = 2, 1
    sig = np.array([1.0, 0.0, 0.0, 1.0])
    d.sigma = sig.ctypes.data
    for k, v in kw.items():
        setattr(d, k, v)
    return d, sig


@pytest.mark.parametrize("field,value,code", [
    ("dim", 4, -1), ("h", 0.0, -1), ("K", 0, -1), ("P", 9, -1), ("scheme", 1, -7), ("coef_model", 3, -7),
    ("restart", 0, -1), ("restart", 65, -1), ("omega", 2.5, -1), ("precision", 5, -1), ("nu1", 0, -1),
    ("rtol_inf", 0.0, -1), ("precond", 7, -1), ("max_levels", -1, -1), ("nu_tight", 17, -1),
    ("coarse_sweeps_t", -1, -1)])
def test_setup_rejects_invalid_arguments(slhjb, field, value, code):
    d, keep = _desc(slhjb, **{field: value})
    h = ctypes.c_void_p()
    rc = slhjb.lib().hjb_setup(ctypes.byref(d), ctypes.byref(h))
    assert rc == code
    assert h.value is None
    assert slhjb.lib().hjb_last_error().decode() != ""


def test_setup_small_axis_and_nonfinite(slhjb):
    d, keep = _desc(slhjb)
    d.n[0] = 2
    h = ctypes.c_void_p()
    assert slhjb.lib().hjb_setup(ctypes.byref(d), ctypes.byref(h)) == -1
    d, keep = _desc(slhjb)
    bad = np.array([np.nan, 0.0, 0.0, 1.0])
    d.sigma = bad.ctypes.data
    assert slhjb.lib().hjb_setup(ctypes.byref(d), ctypes.byref(h)) == -1


def test_setup_without_gpu_reports_device_error(slhjb):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is present")
    d, keep = _desc(slhjb)
    h = ctypes.c_void_p()
    assert slhjb.lib().hjb_setup(ctypes.byref(d), ctypes.byref(h)) == -2
    with pytest.raises(slhjb.HJBError) as e:
        slhjb.Solver(2, (9, 9), (0, 0), 1 / 8, np.eye(2)[:, None, :])
    assert e.value.code == -2


def test_null_handle_calls_fail_cleanly(slhjb):
    L = slhjb.lib()
    st = slhjb.StepStats()
    assert L.hjb_step(None, None, None, None, None, 0.0, 0.1, 1.0, 1.0, None, None, 0.0, ctypes.byref(st)) == -1
    assert L.hjb_profile_enable(None, 0, 10) == -1
    assert L.hjb_profile_sample(None, 4) == -1
    assert L.hjb_apply(None, None, None, None, 0.1, 1.0, 1.0) == -1
    assert L.hjb_apply_transposed(None, None, None, None, 0.1, 1.0, 1.0) == -1
    assert L.hjb_adjoint(None, None, None, None, None, 1, None, None, 1.0, None, None, None, None, None, None, None,
                         None) == -1
    L.hjb_destroy(None)
    assert L.hjb_solve_batch(None, None, None, None, None, 1, None, None, 1.0, None, None, None) == -1
    assert L.hjb_batch_layout(None, None, None) == -1
    assert L.hjb_setup_batch(None, 0, None) == -1
    L.hjb_destroy_batch(None)
    assert L.hjb_set_tile_width(None, 32) == -1
    assert L.hjb_autotune(None, None, None, None) == -1
