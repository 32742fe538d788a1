"""Pins for the oracle's curvatures (CPU only).

Closed forms of a single source (a cone in 2D, spheres in 3D), and on
multi-source fields independent routes to the same quantities: the
fundamental forms and the shape operator of the graph surface (2D); half the
divergence of the unit normal by finite differences, the bordered-Hessian
determinant and the eigenvalues of the tangential Hessian (3D).
"""

import numpy as np
import pytest

import oracle


def _nodes(d, n, seed, lo=0.1, hi=0.9):
    return np.random.default_rng(seed).uniform(lo, hi, (n, d))


def test_cone_closed_form():
    """One source in 2D: S = r, the graph is a 45-degree cone: Gaussian 0,
    mean 1/(2 sqrt2 r), principal 1/(sqrt2 r) and 0."""
    Y = np.array([[0.5, 0.5]])
    X = _nodes(2, 400, 1)
    r = np.linalg.norm(X - Y, axis=1)
    X, r = X[r > 0.05], r[r > 0.05]
    f = oracle.fields(X, Y, 0.01, grad=True, hess=True)
    c = oracle.graph_curvature(f["grad"], f["hess"])
    np.testing.assert_allclose(c["gauss"], 0.0, atol=1e-10)
    np.testing.assert_allclose(c["mean"], 1.0 / (2.0 * np.sqrt(2.0) * r), rtol=1e-10)
    np.testing.assert_allclose(c["k1"], 1.0 / (np.sqrt(2.0) * r), rtol=1e-7)
    np.testing.assert_allclose(c["k2"], 0.0, atol=1e-6 / r.min())


def test_sphere_closed_form():
    """One source in 3D: the level sets are spheres of radius r: mean 1/r,
    Gaussian 1/r^2, both principal curvatures 1/r."""
    Y = np.array([[0.5, 0.5, 0.5]])
    X = _nodes(3, 400, 2)
    r = np.linalg.norm(X - Y, axis=1)
    X, r = X[r > 0.05], r[r > 0.05]
    f = oracle.fields(X, Y, 0.01, grad=True, hess=True)
    c = oracle.level_set_curvature(f["grad"], f["hess"])
    np.testing.assert_allclose(c["mean"], 1.0 / r, rtol=1e-10)
    np.testing.assert_allclose(c["gauss"], 1.0 / r ** 2, rtol=1e-10)
    np.testing.assert_allclose(c["k1"], 1.0 / r, rtol=1e-6)
    np.testing.assert_allclose(c["k2"], 1.0 / r, rtol=1e-6)


def test_plane_and_zero_gradient():
    """A linear S (constant gradient, zero Hessian) is flat; a zero gradient
    gives 0 in 3D (undefined level set) and a flat graph in 2D."""
    g2 = np.tile([0.3, -0.4], (5, 1))
    c = oracle.graph_curvature(g2, np.zeros((5, 2, 2)))
    for k in ("mean", "gauss", "k1", "k2"):
        np.testing.assert_array_equal(c[k], 0.0)
    h3 = np.tile(np.eye(3), (4, 1, 1))
    c = oracle.level_set_curvature(np.zeros((4, 3)), h3)
    for k in ("mean", "gauss", "k1", "k2"):
        np.testing.assert_array_equal(c[k], 0.0)


def _two_sources(d, seed):
    rng = np.random.default_rng(seed)
    Y = rng.uniform(0.35, 0.65, (3, d))
    return Y


@pytest.mark.parametrize("tau", [0.02, 0.05])
def test_graph_fundamental_forms(tau):
    """2D, several sources: K = (L N - M^2)/(E G - F^2) and
    H = (E N - 2 F M + G L)/(2 (E G - F^2)) from the first and second
    fundamental forms of (x, y, S), and k1, k2 as the eigenvalues of the shape
    operator I^-1 II."""
    Y = _two_sources(2, 5)
    X = _nodes(2, 300, 6)
    f = oracle.fields(X, Y, tau, grad=True, hess=True)
    c = oracle.graph_curvature(f["grad"], f["hess"])
    sx, sy = f["grad"][:, 0], f["grad"][:, 1]
    h = f["hess"]
    nrm = np.sqrt(1 + sx ** 2 + sy ** 2)
    E, F, G = 1 + sx ** 2, sx * sy, 1 + sy ** 2
    Lf, Mf, Nf = h[:, 0, 0] / nrm, h[:, 0, 1] / nrm, h[:, 1, 1] / nrm
    den = E * G - F ** 2
    np.testing.assert_allclose(c["gauss"], (Lf * Nf - Mf ** 2) / den, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(c["mean"], (E * Nf - 2 * F * Mf + G * Lf) / (2 * den), rtol=1e-9, atol=1e-9)
    I = np.stack([np.stack([E, F], -1), np.stack([F, G], -1)], -2)
    II = np.stack([np.stack([Lf, Mf], -1), np.stack([Mf, Nf], -1)], -2)
    ev = np.sort(np.linalg.eigvals(np.linalg.solve(I, II)).real, axis=1)
    np.testing.assert_allclose(c["k1"], ev[:, 1], rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(c["k2"], ev[:, 0], rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("tau", [0.02, 0.05])
def test_level_set_independent_routes(tau):
    """3D, several sources: mean curvature = half the divergence of
    grad S / |grad S| (central differences of the oracle's gradient field);
    Gaussian curvature = -det([[H, g], [g^T, 0]]) / |g|^4 (bordered Hessian);
    principal curvatures = the tangential eigenvalues of P H P / |g|."""
    Y = _two_sources(3, 7)
    X = _nodes(3, 200, 8)
    f = oracle.fields(X, Y, tau, grad=True, hess=True)
    g, H = f["grad"], f["hess"]
    keep = np.einsum("ni,ni->n", g, g) > 0.25
    X, g, H = X[keep], g[keep], H[keep]
    c = oracle.level_set_curvature(g, H)
    # divergence of the unit normal by central differences
    dx = 1e-5
    div = np.zeros(len(X))
    for a in range(3):
        e = np.zeros(3)
        e[a] = dx
        gp = oracle.fields(X + e, Y, tau, grad=True)["grad"]
        gm = oracle.fields(X - e, Y, tau, grad=True)["grad"]
        up = gp[:, a] / np.linalg.norm(gp, axis=1)
        um = gm[:, a] / np.linalg.norm(gm, axis=1)
        div += (up - um) / (2 * dx)
    np.testing.assert_allclose(c["mean"], 0.5 * div, rtol=1e-5, atol=1e-4)
    # bordered Hessian
    B = np.zeros((len(X), 4, 4))
    B[:, :3, :3] = H
    B[:, :3, 3] = g
    B[:, 3, :3] = g
    q = np.einsum("ni,ni->n", g, g)
    np.testing.assert_allclose(c["gauss"], -np.linalg.det(B) / q ** 2, rtol=1e-8, atol=1e-8)
    # tangential eigenvalues
    n = g / np.sqrt(q)[:, None]
    P = np.eye(3)[None] - n[:, :, None] * n[:, None, :]
    Ht = P @ H @ P / np.sqrt(q)[:, None, None]
    w, V = np.linalg.eigh(Ht)
    # drop the eigenvalue whose eigenvector is the normal
    normal_idx = np.argmax(np.abs(np.einsum("nij,ni->nj", V, n)), axis=1)
    tang = np.array([np.delete(w[i], normal_idx[i]) for i in range(len(X))])
    np.testing.assert_allclose(c["k1"], tang.max(axis=1), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(c["k2"], tang.min(axis=1), rtol=1e-6, atol=1e-6)
