"""CPU-only checks of the batched plan's host logic: padding rule, argument
validation, and call checks that return before any GPU work."""

import ctypes

import pytest

from tests import parity


@pytest.fixture(scope="module")
def lib():
    from paper_1112_3010_amd import _lib
    return _lib.load()


def _desc(dims_list, tau_h=2.0):
    from paper_1112_3010_amd import _lib
    d = (_lib.DtInstanceDesc * len(dims_list))()
    for i, (nx, ny) in enumerate(dims_list):
        d[i].dims[0], d[i].dims[1] = nx, ny
        d[i].spacing[0], d[i].spacing[1] = 1.0 / nx, 1.0 / ny
        d[i].origin[0], d[i].origin[1] = 0.0, 0.0
        d[i].tau = tau_h / nx
    return d


def _create(lib, dims_list, prec=0, mask=3, ctheta=0.0, desc=None):
    h = ctypes.c_void_p()
    d = desc if desc is not None else _desc(dims_list)
    return lib.dt_create_batch_plan(ctypes.byref(h), len(dims_list), d, prec, mask, ctheta), h


def test_smooth7_rule():
    assert [parity.smooth7_at_least(n) for n in (1, 7, 11, 13, 97, 128, 129, 1000, 1023, 1024)] == \
        [1, 7, 12, 14, 98, 128, 135, 1000, 1024, 1024]
    # brute force: every value is 7-smooth and none smaller in between is
    for n in range(2, 400):
        m = parity.smooth7_at_least(n)
        assert m >= n
        for k in range(n, m):
            r = k
            for p in (2, 3, 5, 7):
                while r % p == 0:
                    r //= p
            assert r != 1


def test_batch_padding_and_offsets(lib):
    from paper_1112_3010_amd import _lib
    dims = [(128, 128), (97, 130), (1000, 37), (1024, 1024), (2, 2)]
    st, h = _create(lib, dims)
    assert st == 0
    off = 0
    for i, (nx, ny) in enumerate(dims):
        info = _lib.DtBatchInstanceInfo()
        assert lib.dt_batch_instance_info(h, i, ctypes.byref(info)) == 0
        assert (info.padded[0], info.padded[1]) == (parity.batch_padded(nx), parity.batch_padded(ny))
        assert info.padded[0] >= 2 * nx - 1 and info.padded[1] >= 2 * ny - 1
        assert info.node_offset == off
        off += nx * ny
        assert info.total_nodes == sum(a * b for a, b in dims)
    size = ctypes.c_size_t()
    assert lib.dt_batch_workspace_size(h, ctypes.byref(size)) == 0 and size.value > 0
    assert lib.dt_destroy_batch_plan(h) == 0


def test_batch_validation(lib):
    assert _create(lib, [(64, 64)])[0] == 0
    assert _create(lib, [(64, 64)], prec=2)[0] == 1          # AUTO is not offered for batches
    assert _create(lib, [(64, 64)], mask=4)[0] == 1          # Hessian is not offered for batches
    assert _create(lib, [(64, 64)], mask=0)[0] == 1
    assert _create(lib, [(1, 64)])[0] == 1
    assert _create(lib, [(64, 2048)])[0] == 6                # DT_E_UNSUPPORTED
    d = _desc([(64, 64)])
    d[0].tau = 0.0
    assert _create(lib, [(64, 64)], desc=d)[0] == 1
    d = _desc([(64, 64)])
    d[0].spacing[1] = float("nan")
    assert _create(lib, [(64, 64)], desc=d)[0] == 1
    h = ctypes.c_void_p()
    assert lib.dt_create_batch_plan(ctypes.byref(h), 0, _desc([(8, 8)]), 0, 1, 0.0) == 1
    assert lib.dt_create_batch_plan(None, 1, _desc([(8, 8)]), 0, 1, 0.0) == 1


def test_batch_call_checks_without_workspace(lib):
    st, h = _create(lib, [(64, 64), (50, 70)])
    assert st == 0
    size = ctypes.c_size_t()
    assert lib.dt_batch_workspace_size(h, ctypes.byref(size)) == 0
    assert lib.dt_batch_set_workspace(h, None, size.value, None) == 1
    assert lib.dt_batch_set_workspace(h, ctypes.c_void_p(4096 + 8), size.value, None) == 4
    assert lib.dt_batch_set_workspace(h, ctypes.c_void_p(4096), 16, None) == 4
    koff = (ctypes.c_int64 * 3)(0, 5, 9)
    dummy = ctypes.c_void_p(4096)
    assert lib.dt_forward_batched(h, dummy, koff, dummy, dummy, None) == 4     # no workspace yet
    assert lib.dt_forward_batched(None, dummy, koff, dummy, dummy, None) == 1
    assert lib.dt_batch_last_error(h) == 1
    from paper_1112_3010_amd import _lib
    t = _lib.DtBatchTiles(8, 256, 256)
    assert lib.dt_batch_set_tiles(h, ctypes.byref(t)) == 0                     # applied at set_workspace
    t2 = _lib.DtBatchTiles()
    assert lib.dt_batch_get_tiles(h, ctypes.byref(t2)) == 0 and t2.col_nb == 8
    assert lib.dt_batch_set_graph(h, 1) == 0
    assert lib.dt_destroy_batch_plan(h) == 0


def test_batch_reduced_padding_rule(lib):
    """k_max > 0: the plan's padded sizes follow the reduced rule, leave room
    for the truncation box (M >= n + c) and never exceed the full padding."""
    from paper_1112_3010_amd import _lib
    dims = [(1024, 1024), (700, 130), (128, 128), (64, 1000), (20, 20)]
    kmax = [20000, 500, 100, 3000, 5]
    for prec, pname in ((0, "fp32"), (1, "fp64")):
        d = _desc(dims)
        for i, k in enumerate(kmax):
            d[i].k_max = k
        st, h = _create(lib, dims, prec=prec, desc=d)
        assert st == 0
        reduced_any = False
        for i, (nx, ny) in enumerate(dims):
            info = _lib.DtBatchInstanceInfo()
            assert lib.dt_batch_instance_info(h, i, ctypes.byref(info)) == 0
            Ms, cuts = parity.batch_padded_reduced((nx, ny), (1.0 / nx, 1.0 / ny), 2.0 / nx, kmax[i], pname)
            assert (info.padded[0], info.padded[1]) == Ms, (pname, i)
            for n, M, c in zip((nx, ny), Ms, cuts):
                assert M <= parity.batch_padded(n)
                if c:
                    assert M >= n + c
                    reduced_any = True
        assert reduced_any
        # the 1024^2 instance shrinks from 2048 per axis
        info = _lib.DtBatchInstanceInfo()
        assert lib.dt_batch_instance_info(h, 0, ctypes.byref(info)) == 0
        assert info.padded[0] < 2048 and info.padded[1] < 2048
        assert lib.dt_destroy_batch_plan(h) == 0
    d = _desc([(64, 64)])
    d[0].k_max = -1
    assert _create(lib, [(64, 64)], desc=d)[0] == 1
