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
    # beyond the float64 band: double-double (band about 60 tau here), then
    # quad-double (about 130 tau), then no precision resolves it
    for trunc, want in ((40, 3), (80, 4)):
        st, h = _plan(lib, dims=dims, tau=tau, prec=2, mask=1, trunc=trunc * tau, khint=1000)
        assert st == 0
        assert lib.dt_plan_info(h, ctypes.byref(info)) == 0
        assert info.precision == want, (trunc, info.precision)
        lib.dt_destroy_plan(h)
    assert _plan(lib, dims=dims, tau=tau, prec=2, mask=1, trunc=200 * tau, khint=1000)[0] == 3
    # quad-double is not offered for the sign (as double-double)
    assert _plan(lib, dims=dims, tau=tau, prec=4, mask=8)[0] == 6


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


def test_static_workspace_refuses_large_plans(lib):
    """The fixed workspace array holds DT_STATIC_WORKSPACE_BYTES; a plan that
    needs more is refused on the host before any device call."""
    assert lib.dt_plan_set_static_workspace(None, None) == 1
    st, h = _plan(lib, ndim=3, dims=(256, 256, 256), tau=1.0 / 256)
    assert st == 0
    size = ctypes.c_size_t()
    assert lib.dt_plan_workspace_size(h, ctypes.byref(size)) == 0
    from paper_1112_3010_amd import _lib
    assert size.value > _lib.DT_STATIC_WORKSPACE_BYTES
    assert lib.dt_plan_set_static_workspace(h, None) == 4
    assert lib.dt_distance(h, ctypes.c_void_p(4096), 10, ctypes.c_void_p(4096), None) == 4   # still no workspace
    assert lib.dt_destroy_plan(h) == 0


def test_struct_layouts_match_header(tmp_path):
    """Every public struct of include/dt.h has the same size and field
    offsets in C (compiled here with gcc against the header) as in the
    ctypes mirrors of the Python binding."""
    import shutil
    import subprocess
    from paper_1112_3010_amd import _lib
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = {
        "dt_shape": _lib.DtShape, "dt_outputs": _lib.DtOutputs, "dt_plan_info_t": _lib.DtPlanInfo,
        "dt_call_stats": _lib.DtCallStats, "dt_pass_timing": _lib.DtPassTiming,
        "dt_instance_desc": _lib.DtInstanceDesc, "dt_batch_instance_info_t": _lib.DtBatchInstanceInfo,
        "dt_batch_tiles": _lib.DtBatchTiles,
    }
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dt.h"', "int main(void) {"]
    for cname, cls in pairs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, *_ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln.strip():
            cname, key, val = ln.split()
            got[(cname, key)] = int(val)
    for cname, cls in pairs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, *_ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_fp64x2_plans(lib):
    from paper_1112_3010_amd import _lib
    st, h = _plan(lib, prec=3, mask=1)
    assert st == 0
    info = _lib.DtPlanInfo()
    assert lib.dt_plan_info(h, ctypes.byref(info)) == 0
    assert info.precision == 3 and info.unit_roundoff == 2.0 ** -104
    size = ctypes.c_size_t()
    assert lib.dt_plan_workspace_size(h, ctypes.byref(size)) == 0
    assert size.value >= 128 * 128 * (32 + 16)          # complex grid + real spectrum
    dummy = ctypes.c_void_p(4096)
    assert lib.dt_distance(h, dummy, 10, dummy, None) == 4          # no workspace yet
    assert lib.dt_gradient(h, dummy, 10, None, dummy, None) == 1    # no gradient kernels
    assert lib.dt_backward(h, dummy, 10, dummy, dummy, dummy, None, None) == 1
    lib.dt_destroy_plan(h)
    st, h = _plan(lib, prec=3, mask=3)                               # S and grad S
    assert st == 0
    lib.dt_destroy_plan(h)
    st, h = _plan(lib, prec=3, mask=5)                               # S and the Hessian
    assert st == 0
    assert lib.dt_hessian(h, dummy, 10, dummy, None) == 4            # no workspace yet
    lib.dt_destroy_plan(h)
    st, h = _plan(lib, prec=3, mask=1 | 32)                          # S and curvatures
    assert st == 0
    lib.dt_destroy_plan(h)
    st, h = _plan(lib, prec=3, mask=1 | 16)                          # S and the adjoint
    assert st == 0
    lib.dt_destroy_plan(h)
    assert _plan(lib, prec=3, mask=1 | 8)[0] == 6                    # the sign channels are not built
    st, h = _plan(lib, ndim=3, dims=(32, 32, 30), prec=3, mask=3)    # 3D S and grad S
    assert st == 0
    assert lib.dt_plan_info(h, ctypes.byref(info)) == 0
    assert info.precision == 3 and tuple(info.padded[:3]) == (64, 64, 64)
    assert lib.dt_plan_workspace_size(h, ctypes.byref(size)) == 0
    # four spectra (f and three gradient kernels), the complex work grids
    assert size.value >= 64 ** 3 * (4 * 16 + 32)
    lib.dt_destroy_plan(h)
    assert _plan(lib, ndim=3, dims=(257, 32, 32), prec=3, mask=1)[0] == 6   # 3D up to 256 per axis
    assert _plan(lib, ndim=3, dims=(32, 32, 32), prec=3, mask=9)[0] == 6    # no sign channels


def test_auto_picks_fp64x2_for_2d_distance(lib):
    from paper_1112_3010_amd import _lib
    dims = (128, 128)
    tau = 2.0 / 128
    st, h = _plan(lib, dims=dims, tau=tau, prec=2, mask=1, trunc=45 * tau, khint=1000)
    assert st == 0
    info = _lib.DtPlanInfo()
    assert lib.dt_plan_info(h, ctypes.byref(info)) == 0
    assert info.precision == 3
    lib.dt_destroy_plan(h)
    # with the Hessian too; with the sign channels there is no extended-precision candidate
    st, h = _plan(lib, dims=dims, tau=tau, prec=2, mask=5, trunc=45 * tau, khint=1000)
    assert st == 0 and lib.dt_plan_info(h, ctypes.byref(info)) == 0 and info.precision == 3
    lib.dt_destroy_plan(h)
    assert _plan(lib, dims=dims, tau=tau, prec=2, mask=1 | 8, trunc=45 * tau, khint=1000)[0] == 3


def _reduced(lib, dims, tau, k_max, prec=0, mask=3, ndim=None):
    h = ctypes.c_void_p()
    nd = ndim or len(dims)
    d = (ctypes.c_int64 * len(dims))(*dims)
    sp = (ctypes.c_double * len(dims))(*[1.0 / n for n in dims])
    org = (ctypes.c_double * len(dims))(*([0.0] * len(dims)))
    return lib.dt_create_plan_reduced(ctypes.byref(h), nd, d, sp, org, tau, prec, mask, k_max, 0.0), h


@pytest.mark.parametrize("dims,tau_cells,k_max,prec", [
    ((200, 200, 200), 2.0, 2000, 0), ((160, 160, 160), 2.0, 2000, 1), ((300, 130, 90), 1.5, 64, 0),
    ((1000, 1000), 1.0, 5000, 0), ((100, 100), 20.0, 100, 0), ((640, 96), 2.5, 1, 1)])
def test_reduced_padding_rule(lib, dims, tau_cells, k_max, prec):
    """The library's reduced padded sizes and truncation boxes follow the
    documented rule (recomputed in tests/parity.py)."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import parity
    from paper_1112_3010_amd import _lib
    tau = tau_cells / dims[0]
    st, h = _reduced(lib, dims, tau, k_max, prec)
    assert st == 0
    info = _lib.DtPlanInfo()
    assert lib.dt_plan_info(h, ctypes.byref(info)) == 0
    Mp, cut = parity.padded_reduced(dims, [1.0 / n for n in dims], tau, k_max, "fp64" if prec else "fp32")
    D = len(dims)
    assert tuple(info.padded[:D]) == Mp and tuple(info.cut[:D]) == cut and info.k_max == k_max
    full = tuple(parity.padded(n) for n in dims)
    assert all(m <= f for m, f in zip(Mp, full))
    for m, n, c in zip(Mp, dims, cut):
        assert m >= 64 and (m & (m - 1) == 0 or m in (288, 392))
        assert c == 0 or m >= n + c
    lib.dt_destroy_plan(h)


def test_reduced_padding_shrinks_and_refuses(lib):
    from paper_1112_3010_amd import _lib
    # 160^3 with tau = 2 cells and 2000 sources: 512^3 -> 256^3
    st, h = _reduced(lib, (160, 160, 160), 2.0 / 160, 2000)
    assert st == 0
    info = _lib.DtPlanInfo()
    assert lib.dt_plan_info(h, ctypes.byref(info)) == 0
    assert tuple(info.padded[:3]) == (256, 256, 256) and all(0 < c <= 96 for c in info.cut[:3])
    dummy = ctypes.c_void_p(4096)
    # a call with more sources than k_max is refused before any device work
    assert lib.dt_distance(h, dummy, 2001, dummy, None) == 1
    lib.dt_destroy_plan(h)
    assert _reduced(lib, (64, 64), 0.03, 0)[0] == 1                  # k_max >= 1
    assert _reduced(lib, (64, 64), 0.03, 10, prec=2)[0] == 1         # AUTO
    assert _reduced(lib, (64, 64), 0.03, 10, prec=3)[0] == 1         # double-double
    assert _reduced(lib, (64, 64), 0.03, 10, mask=1 | 8)[0] == 6     # sign kernels do not decay
    # a wide kernel keeps the full padding, untruncated
    st, h = _reduced(lib, (100, 100), 0.5, 10)
    assert st == 0 and lib.dt_plan_info(h, ctypes.byref(info)) == 0
    assert tuple(info.padded[:2]) == (256, 256) and tuple(info.cut[:2]) == (0, 0)
    lib.dt_destroy_plan(h)
