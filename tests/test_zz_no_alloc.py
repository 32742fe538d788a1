"""The allocation-free attach, dt_plan_set_static_workspace, against the
ordinary one, dt_plan_set_workspace, through the C ABI.

Both run the same kernels on the same inputs; only the workspace differs
(the library's fixed per-device array instead of caller memory), so S,
grad S and the validity scalars must agree bit for bit.  Two attaches in a
row, the second with a smaller grid, check that the array is reused and
that the earlier holder is refused afterwards."""

import ctypes

import numpy as np
import pytest
import torch

import synth
from paper_1112_3010_amd import _lib as L

pytestmark = pytest.mark.gpu


def _create(lib, dims, tau, prec):
    h = ctypes.c_void_p()
    n = len(dims)
    d = (ctypes.c_int64 * n)(*dims)
    sp = (ctypes.c_double * n)(*[1.0 / x for x in dims])
    org = (ctypes.c_double * n)(*([0.0] * n))
    L.check(lib.dt_create_plan(ctypes.byref(h), n, d, sp, org, tau, prec, L.DT_OUT_S | L.DT_OUT_GRAD, 0.0, 0, 0.0),
            "dt_create_plan")
    return h


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _gradient(lib, h, Y, dims, dtype):
    shape = tuple(reversed(dims))
    S = torch.full(shape, float("nan"), dtype=dtype, device="cuda")
    g = torch.full((len(dims), *shape), float("nan"), dtype=dtype, device="cuda")
    st = lib.dt_gradient(h, ctypes.c_void_p(Y.data_ptr()), Y.shape[0], ctypes.c_void_p(S.data_ptr()),
                         ctypes.c_void_p(g.data_ptr()), _stream())
    L.check(st, "dt_gradient")
    stats = L.DtCallStats()
    L.check(lib.dt_last_stats(h, ctypes.byref(stats)), "dt_last_stats")
    torch.cuda.synchronize()
    return S.cpu().numpy(), g.cpu().numpy(), (stats.theta, stats.s_max, stats.g_l2)


# (grid, tau in cells, precision, sources, seed); the second grid is the smaller one
CASES = [((40, 36, 33), 1.5, L.DT_FP32_SCALED, torch.float32, 200, 231),
         ((96, 80), 2.0, L.DT_FP64, torch.float64, 40, 17)]


def test_static_workspace_matches_caller_workspace():
    lib = L.load()
    torch.cuda.init()
    held = []
    for dims, tau_cells, prec, dtype, K, seed in CASES:
        print(f"static workspace: grid {dims}, precision {prec}, K {K}", flush=True)
        tau = tau_cells / dims[0]
        Y = torch.from_numpy(synth.generators.uniform_points(len(dims), K, seed=seed)).cuda()

        ref_h = _create(lib, dims, tau, prec)
        size = ctypes.c_size_t()
        L.check(lib.dt_plan_workspace_size(ref_h, ctypes.byref(size)), "dt_plan_workspace_size")
        assert size.value <= L.DT_STATIC_WORKSPACE_BYTES
        ws = torch.empty(size.value + 256, dtype=torch.uint8, device="cuda")
        base = ws.data_ptr() + (-ws.data_ptr()) % 256
        L.check(lib.dt_plan_set_workspace(ref_h, ctypes.c_void_p(base), size.value, _stream()),
                "dt_plan_set_workspace")
        S_ref, g_ref, st_ref = _gradient(lib, ref_h, Y, dims, dtype)

        h = _create(lib, dims, tau, prec)
        L.check(lib.dt_plan_set_static_workspace(h, _stream()), "dt_plan_set_static_workspace")
        # an earlier holder of the array is refused once this plan has taken it
        # over (with inputs and outputs sized for that holder, so that the call
        # would stay in bounds even if it were enqueued)
        for old, old_dims, old_dtype, old_K in held:
            Y_old = torch.full((old_K, len(old_dims)), 0.5, dtype=torch.float32, device="cuda")
            S_old = torch.empty(tuple(reversed(old_dims)), dtype=old_dtype, device="cuda")
            assert lib.dt_distance(old, ctypes.c_void_p(Y_old.data_ptr()), old_K, ctypes.c_void_p(S_old.data_ptr()),
                                   _stream()) == L.DT_E_WORKSPACE
            assert lib.dt_last_error(old) == L.DT_E_WORKSPACE
        S, g, st = _gradient(lib, h, Y, dims, dtype)
        # twice in a row on the same array: the second call starts from the
        # first call's leftovers and must clear what it needs
        S2, g2, st2 = _gradient(lib, h, Y, dims, dtype)
        assert lib.dt_last_error(h) == L.DT_OK

        assert np.isfinite(S_ref).all() and np.isfinite(g_ref).all()
        assert np.array_equal(S, S_ref) and np.array_equal(g, g_ref)
        assert np.array_equal(S2, S_ref) and np.array_equal(g2, g_ref)
        assert st == st_ref and st2 == st_ref
        lib.dt_destroy_plan(ref_h)
        del ws
        held.append((h, dims, dtype, K))

    # the first plan works again once it is attached again
    dims, tau_cells, prec, dtype, K, seed = CASES[0]
    Y = torch.from_numpy(synth.generators.uniform_points(len(dims), K, seed=seed)).cuda()
    first = held[0][0]
    L.check(lib.dt_plan_set_static_workspace(first, _stream()), "dt_plan_set_static_workspace")
    S_again, _, _ = _gradient(lib, first, Y, dims, dtype)
    assert lib.dt_last_error(held[1][0]) == L.DT_E_WORKSPACE
    ref = _create(lib, dims, tau_cells / dims[0], prec)
    size = ctypes.c_size_t()
    L.check(lib.dt_plan_workspace_size(ref, ctypes.byref(size)), "dt_plan_workspace_size")
    ws = torch.empty(size.value + 256, dtype=torch.uint8, device="cuda")
    base = ws.data_ptr() + (-ws.data_ptr()) % 256
    L.check(lib.dt_plan_set_workspace(ref, ctypes.c_void_p(base), size.value, _stream()), "dt_plan_set_workspace")
    S_ref, _, _ = _gradient(lib, ref, Y, dims, dtype)
    assert np.array_equal(S_again, S_ref)
    for h in [x[0] for x in held] + [ref]:
        lib.dt_destroy_plan(h)


def test_static_workspace_refuses_oversized_plan():
    lib = L.load()
    h = _create(lib, (128, 128, 128), 1.0 / 128, L.DT_FP32_SCALED)
    assert lib.dt_plan_set_static_workspace(h, _stream()) == L.DT_E_WORKSPACE
    lib.dt_destroy_plan(h)
