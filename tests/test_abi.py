"""CPU-only checks of the C ABI: the library loads, exports every function
that include/dt.h declares, and rejects bad arguments on the host (no GPU
call is made by any of these paths)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dt.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1112_3010_amd import _lib
    return _lib.load()


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const char\*|dt_status)\s+(dt_\w+)\s*\(", text, re.M)))


def test_header_declarations_exported(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    from paper_1112_3010_amd import _lib
    assert set(names) == set(_lib.EXPORTED)


def _plan(lib, ndim=2, dims=(64, 64), tau=0.03, prec=0, mask=3, trunc=0.0, khint=0, ctheta=0.0):
    h = ctypes.c_void_p()
    d = (ctypes.c_int64 * len(dims))(*dims)
    sp = (ctypes.c_double * len(dims))(*[1.0 / n for n in dims])
    org = (ctypes.c_double * len(dims))(*([0.0] * len(dims)))
    st = lib.dt_create_plan(ctypes.byref(h), ndim, d, sp, org, tau, prec, mask, trunc, khint, ctheta)
    return st, h


def test_create_plan_validation(lib):
    assert _plan(lib)[0] == 0
    assert _plan(lib, ndim=4, dims=(8, 8, 8, 8))[0] == 1
    assert _plan(lib, tau=0.0)[0] == 1
    assert _plan(lib, tau=float("nan"))[0] == 1
    assert _plan(lib, dims=(1, 64))[0] == 1
    assert _plan(lib, prec=7)[0] == 1
    assert _plan(lib, mask=0)[0] == 1
    assert _plan(lib, mask=1 << 9)[0] == 1
    assert _plan(lib, dims=(2048, 64))[0] == 6          # DT_E_UNSUPPORTED
    assert _plan(lib, prec=2)[0] == 1                   # AUTO needs k_hint
    assert lib.dt_create_plan(None, 2, None, None, None, 0.1, 0, 1, 0.0, 0, 0.0) == 1


def test_auto_precision(lib):
    from paper_1112_3010_amd import _lib
    dims = (128, 128)
    tau = 2.0 / 128
    st, h = _plan(lib, dims=dims, tau=tau, prec=2, mask=1, trunc=3 * tau, khint=1000)
    assert st == 0
    info = _lib.DtPlanInfo()
    assert lib.dt_plan_info(h, ctypes.byref(info)) == 0
    assert info.precision == 0 and tuple(info.padded[:2]) == (256, 256)
    lib.dt_destroy_plan(h)
    st, h = _plan(lib, dims=dims, tau=tau, prec=2, mask=1, trunc=20 * tau, khint=1000)
    assert st == 0
    assert lib.dt_plan_info(h, ctypes.byref(info)) == 0
    assert info.precision == 1
    lib.dt_destroy_plan(h)
    assert _plan(lib, dims=dims, tau=tau, prec=2, mask=1, trunc=80 * tau, khint=1000)[0] == 3


def test_workspace_and_call_checks(lib):
    st, h = _plan(lib)
    assert st == 0
    size = ctypes.c_size_t()
    assert lib.dt_plan_workspace_size(h, ctypes.byref(size)) == 0 and size.value > 0
    assert lib.dt_plan_set_workspace(h, None, size.value, None) == 1
    assert lib.dt_plan_set_workspace(h, ctypes.c_void_p(4096 + 8), size.value, None) == 4
    assert lib.dt_plan_set_workspace(h, ctypes.c_void_p(4096), 16, None) == 4
    dummy = ctypes.c_void_p(4096)
    assert lib.dt_distance(h, dummy, 0, dummy, None) == 1          # K = 0
    assert lib.dt_distance(h, dummy, 10, dummy, None) == 4         # no workspace yet
    assert lib.dt_distance(None, dummy, 10, dummy, None) == 1
    assert lib.dt_hessian(h, dummy, 10, dummy, None) == 1          # plan has no Hessian kernels
    assert lib.dt_backward(h, dummy, 10, dummy, dummy, dummy, None, None) == 1   # no backward kernels
    assert lib.dt_sign(h, None, None, None, None) == 1
    assert lib.dt_status_str(2) == b"a source was outside the grid or non-finite"
    assert lib.dt_destroy_plan(h) == 0
