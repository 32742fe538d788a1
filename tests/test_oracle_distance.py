"""Pins for the oracle's distance, gradient and Hessian (CPU only).

Each check compares the oracle with something other than itself: the
paper's error bracket, closed forms, a KD-tree, an FFT convolution done by
scipy, and finite differences.
"""

import numpy as np
import pytest

import oracle
import synth


def _random_case(seed, d=2, k=40, n=64):
    rng = np.random.default_rng(seed)
    Y = rng.random((k, d))
    X = rng.random((300, d))
    return X, Y


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("tau", [0.002, 0.01, 0.05])
def test_error_bracket(d, tau):
    """R - tau log K <= S <= R at every node (Sec. 2.4, eqs. Bound1, errorBound)."""
    X, Y = _random_case(d * 7 + int(tau * 1e4), d=d)
    f = oracle.fields(X, Y, tau)
    K = len(Y)
    assert np.all(f["S"] <= f["R"] + 1e-15)
    assert np.all(f["S"] >= f["R"] - tau * np.log(K) - 1e-15)


def test_nearest_matches_kdtree():
    """R by brute force equals a KD-tree nearest-neighbour query (Sec. 1, eq. Rdef)."""
    from scipy.spatial import cKDTree
    X, Y = _random_case(3, d=3, k=500)
    R = oracle.nearest_distance(X, Y)
    dk, _ = cKDTree(Y).query(X)
    np.testing.assert_allclose(R, dk, rtol=0, atol=1e-15)
    np.testing.assert_allclose(oracle.fields(X, Y, 0.01)["R"], dk, rtol=0, atol=1e-15)


def test_single_source_is_exact():
    """K = 1: S = R, grad S = unit vector, H = (I - n n^T)/r."""
    rng = np.random.default_rng(4)
    X = rng.random((50, 3))
    Y = np.array([[0.31, 0.52, 0.47]])
    f = oracle.fields(X, Y, 0.03, hess=True)
    diff = X - Y
    r = np.linalg.norm(diff, axis=1)
    n = diff / r[:, None]
    np.testing.assert_allclose(f["S"], r, rtol=0, atol=1e-14)
    np.testing.assert_allclose(f["grad"], n, rtol=0, atol=1e-14)
    H = (np.eye(3)[None] - n[:, :, None] * n[:, None, :]) / r[:, None, None]
    np.testing.assert_allclose(f["hess"], H, rtol=1e-12, atol=1e-10)


def test_coincident_sources_multiplicity():
    """m coincident sources: S = R - tau log m exactly."""
    X = np.random.default_rng(5).random((20, 2))
    Y = np.repeat([[0.4, 0.6]], 5, axis=0)
    tau = 0.02
    f = oracle.fields(X, Y, tau)
    np.testing.assert_allclose(f["S"], np.linalg.norm(X - Y[0], axis=1) - tau * np.log(5), atol=1e-14)


def test_monotone_in_tau():
    """S increases as tau decreases (Sec. 2.4); non-strict because of K = 1 and
    exact ties."""
    X, Y = _random_case(6, d=2, k=30)
    taus = [0.001, 0.003, 0.01, 0.03, 0.1]
    S = [oracle.fields(X, Y, t)["S"] for t in taus]
    for a, b in zip(S, S[1:]):
        assert np.all(a >= b - 1e-14)


def test_lse_equals_literal_sum():
    """The log-sum-exp evaluation equals the literal printed form of eq. STilde
    where the literal form does not underflow."""
    X, Y = _random_case(7, d=3, k=60)
    for tau in (0.02, 0.1):
        np.testing.assert_allclose(oracle.fields(X, Y, tau)["S"], oracle.distance_literal(X, Y, tau),
                                   rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("dims", [(48, 40), (20, 18, 16)])
def test_direct_sum_equals_scipy_fft_convolution(dims):
    """The direct sum equals the paper's Table 1 algorithm carried out with
    scipy's FFT in float64 (zero-padded), node by node, for a moderate tau."""
    D = len(dims)
    h = tuple(1.0 / n for n in dims)
    pts = synth.random_grid_points(dims, 25, seed=11 + D)
    idx, valid = oracle.snap(pts, (0.0,) * D, h, dims)
    assert valid.all()
    tau = 2.0 * h[0]
    S_fft = oracle.table1_distance(idx, dims, h, tau)
    X = oracle.grid_nodes(dims, (0.0,) * D, h)
    Yh = oracle.node_coords(idx, (0.0,) * D, h)
    S = oracle.fields(X, Yh, tau)["S"].reshape(S_fft.shape)
    np.testing.assert_allclose(S, S_fft, rtol=1e-9, atol=1e-12)


def _fd_grad(X, Y, tau, step):
    D = X.shape[1]
    g = np.empty_like(X)
    for d in range(D):
        e = np.zeros(D)
        e[d] = step
        g[:, d] = (oracle.fields(X + e, Y, tau)["S"] - oracle.fields(X - e, Y, tau)["S"]) / (2 * step)
    return g


@pytest.mark.parametrize("d", [2, 3])
def test_gradient_matches_finite_differences(d):
    """grad S (Sec. 5, eq. SxSy) against central differences of S."""
    rng = np.random.default_rng(8 + d)
    Y = rng.random((25, d))
    X = rng.random((200, d))
    X = X[oracle.nearest_distance(X, Y) > 0.02]
    tau = 0.02
    g = oracle.fields(X, Y, tau, grad=True)["grad"]
    np.testing.assert_allclose(g, _fd_grad(X, Y, tau, 1e-6), atol=2e-7)


@pytest.mark.parametrize("d", [2, 3])
def test_hessian_matches_finite_differences(d):
    """The Hessian against central differences of the analytic gradient."""
    rng = np.random.default_rng(9 + d)
    Y = rng.random((20, d))
    X = rng.random((150, d))
    X = X[oracle.nearest_distance(X, Y) > 0.03]
    tau = 0.03
    H = oracle.fields(X, Y, tau, hess=True)["hess"]
    step = 1e-6
    for j in range(d):
        e = np.zeros(d)
        e[j] = step
        gp = oracle.fields(X + e, Y, tau, grad=True)["grad"]
        gm = oracle.fields(X - e, Y, tau, grad=True)["grad"]
        np.testing.assert_allclose(H[:, :, j], (gp - gm) / (2 * step), rtol=1e-5, atol=1e-4)
    np.testing.assert_allclose(H, np.swapaxes(H, 1, 2), atol=1e-9)


def test_hessian_2d_matches_printed_formulas():
    """In 2D the general Hessian equals eqs. Sxx, Syy, Sxy of Sec. 5 written
    with f_c = x/r, f_s = y/r, f_r = 1/r."""
    rng = np.random.default_rng(13)
    Y = rng.random((15, 2))
    X = rng.random((100, 2))
    X = X[oracle.nearest_distance(X, Y) > 1e-3]
    tau = 0.05
    f = oracle.fields(X, Y, tau, hess=True)
    d = X[:, None, :] - Y[None]
    r = np.linalg.norm(d, axis=2)
    fc, fs, fr, ff = d[..., 0] / r, d[..., 1] / r, 1 / r, np.exp(-r / tau)
    phi = ff.sum(1)
    Sx, Sy = (fc * ff).sum(1) / phi, (fs * ff).sum(1) / phi
    Sxx = ((-fc ** 2 / tau + fs ** 2 * fr) * ff).sum(1) / phi + Sx ** 2 / tau
    Syy = ((-fs ** 2 / tau + fc ** 2 * fr) * ff).sum(1) / phi + Sy ** 2 / tau
    Sxy = (-(1 / tau + fr) * fc * fs * ff).sum(1) / phi + Sx * Sy / tau
    np.testing.assert_allclose(f["hess"][:, 0, 0], Sxx, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(f["hess"][:, 1, 1], Syy, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(f["hess"][:, 0, 1], Sxy, rtol=1e-9, atol=1e-9)


def test_gradient_norm_below_one():
    """||grad S|| <= 1 everywhere and < 1 where several directions carry
    weight (Sec. 5.1)."""
    rng = np.random.default_rng(14)
    Y = rng.random((30, 3))
    X = rng.random((400, 3))
    f = oracle.fields(X, Y, 0.05, grad=True)
    norm = np.linalg.norm(f["grad"], axis=1)
    assert np.all(norm <= 1 + 1e-12)
    assert np.all(norm < 1)


def test_rmean_gives_tau_derivative():
    """dS/dtau = (S - <r>)/tau against a central difference in tau, and
    dS/dtau <= 0 (S increases as tau decreases, Sec. 2.4)."""
    X, Y = _random_case(15, d=3, k=30)
    tau = 0.04
    f = oracle.fields(X, Y, tau, rmean=True)
    dtau = (f["S"] - f["rmean"]) / tau
    step = 1e-6
    fd = (oracle.fields(X, Y, tau + step)["S"] - oracle.fields(X, Y, tau - step)["S"]) / (2 * step)
    np.testing.assert_allclose(dtau, fd, rtol=1e-6, atol=1e-8)
    assert np.all(dtau <= 1e-15)


def test_snap_rule():
    """Cell-centred snapping: floor((y - o)/h); a point on a face goes to the
    upper cell; outside points are rejected."""
    pts = np.array([[0.0, 0.0], [0.5, 0.25], [0.999, 0.001], [1.0, 0.5], [-1e-7, 0.5], [np.nan, 0.1]],
                   dtype=np.float32)
    idx, valid = oracle.snap(pts, (0.0, 0.0), (0.25, 0.25), (4, 4))
    assert valid.tolist() == [True, True, True, False, False, False]
    assert idx[:3].tolist() == [[0, 0], [2, 1], [3, 0]]
    np.testing.assert_allclose(oracle.node_coords(idx[:3], (0, 0), (0.25, 0.25)),
                               [[0.125, 0.125], [0.625, 0.375], [0.875, 0.125]])
