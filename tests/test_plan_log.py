"""CPU checks of the plan log: with DT_LOG set, plan creation prints the
padded grid, the engines and the tables to stderr; without it nothing is
printed.  (The attach and per-call lines need a device: tests/test_gpu_log.py.)"""

import ctypes
import re

import pytest


@pytest.fixture(scope="module")
def lib():
    from paper_1112_3010_amd import _lib
    return _lib.load()


def _create(lib, dims, tau_cells, prec, mask=3, k_max=0):
    n = len(dims)
    h = ctypes.c_void_p()
    d = (ctypes.c_int64 * n)(*dims)
    sp = (ctypes.c_double * n)(*[1.0 / v for v in dims])
    org = (ctypes.c_double * n)(*([0.0] * n))
    tau = tau_cells / dims[0]
    if k_max:
        st = lib.dt_create_plan_reduced(ctypes.byref(h), n, d, sp, org, tau, prec, mask, k_max, 0.0)
    else:
        st = lib.dt_create_plan(ctypes.byref(h), n, d, sp, org, tau, prec, mask, 0.0, 0, 0.0)
    assert st == 0
    return h


def _lines(err):
    return [l for l in err.splitlines() if l.startswith("[dt] ")]


def test_no_output_without_dt_log(lib, capfd, monkeypatch):
    monkeypatch.delenv("DT_LOG", raising=False)
    h = _create(lib, (64, 48), 2.0, 0)
    lib.dt_destroy_plan(h)
    monkeypatch.setenv("DT_LOG", "0")
    h = _create(lib, (64, 48), 2.0, 0)
    lib.dt_destroy_plan(h)
    assert _lines(capfd.readouterr().err) == []


def test_full_plan_3d(lib, capfd, monkeypatch):
    monkeypatch.setenv("DT_LOG", "1")
    h = _create(lib, (256, 256, 256), 1.0, 0)
    lib.dt_destroy_plan(h)
    out = "\n".join(_lines(capfd.readouterr().err))
    assert "3D grid 256x256x256" in out and "precision fp32-scaled (u = 2^-24)" in out
    assert "outputs S|grad" in out and "c_theta = 256" in out
    assert "padded 512x512x512 (full zero padding)" in out
    # rows: 256-point complex transforms of radices 8, 4, 8
    assert re.search(r"rows R2C / C2R of 512 points \(256-point complex, radices 8x4x8, 8 points per thread\)", out)
    assert "fused z pass" in out and "tables: f u_x u_y u_z (4 of" in out


def test_reduced_plan_reports_cut(lib, capfd, monkeypatch):
    from paper_1112_3010_amd import _lib
    monkeypatch.setenv("DT_LOG", "1")
    h = _create(lib, (256, 256, 256), 1.0, 1, k_max=60000)
    info = _lib.DtPlanInfo()
    assert lib.dt_plan_info(h, ctypes.byref(info)) == 0
    lib.dt_destroy_plan(h)
    out = "\n".join(_lines(capfd.readouterr().err))
    M = "x".join(str(v) for v in info.padded[:3])
    cut = "x".join(str(v) for v in info.cut[:3])
    assert f"padded {M}, reduced for at most 60000 sources: kernels truncated to {cut} cells" in out
    assert "precision fp64" in out


def test_extended_and_batch_plans(lib, capfd, monkeypatch):
    from tests.test_batch_host import _desc
    monkeypatch.setenv("DT_LOG", "1")
    h = _create(lib, (128, 96), 2.0, 3, mask=1)
    lib.dt_destroy_plan(h)
    h = _create(lib, (64, 40, 36), 2.0, 4, mask=3)
    lib.dt_destroy_plan(h)
    hb = ctypes.c_void_p()
    assert lib.dt_create_batch_plan(ctypes.byref(hb), 2, _desc([(128, 200), (97, 64)]), 1, 3, 0.0) == 0
    lib.dt_destroy_batch_plan(hb)
    out = "\n".join(_lines(capfd.readouterr().err))
    assert "precision fp64x2 (u = 2^-104)" in out and "double-double radix-2" in out
    assert "precision fp64x4 (u = 2^-208)" in out and "quad-double radix-2" in out
    assert "batch plan" in out and "2 2D instances, precision fp64" in out
    # the batched padding: 2 x the 7-smooth length at least n along x, 2 x that of n along y
    assert "inst 0: grid 128x200" in out and "padded 256x400" in out
    assert "inst 1: grid 97x64" in out and "padded 196x128" in out
