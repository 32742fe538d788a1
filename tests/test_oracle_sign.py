"""Pins for the oracle's winding number, topological degree and the exact
geometric inside/outside and distance routines (CPU only)."""

import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("K", [3, 4, 7, 24, 200])
def test_regular_polygon_closed_form(K):
    """For a regular K-gon centred on X, every term of eq. kappdiscreteZ equals
    sin(2 pi/K), so mu = K sin(2 pi/K)/(2 pi) exactly; it tends to 1."""
    c = np.array([0.37, 0.61])
    poly = synth.generators.regular_polygon(K, 0.21, c, phase=0.3)
    mu = oracle.winding_number(c[None], poly)[0]
    assert mu == pytest.approx(K * np.sin(2 * np.pi / K) / (2 * np.pi), rel=1e-13)


def test_winding_orientation_and_outside():
    """Counter-clockwise curves wind +1 around inner points, clockwise -1,
    and 0 around outer points (Sec. 4.1)."""
    c = np.array([0.5, 0.5])
    poly = synth.generators.regular_polygon(4000, 0.3, c)
    X = np.array([[0.5, 0.5], [0.55, 0.45], [0.95, 0.5], [0.1, 0.1]])
    mu = oracle.winding_number(X, poly)
    np.testing.assert_allclose(mu, [1, 1, 0, 0], atol=1e-4)
    np.testing.assert_allclose(oracle.winding_number(X, poly[::-1]), [-1, -1, 0, 0], atol=1e-4)


def test_discrete_winding_approaches_exact_winding():
    """Far from a finely sampled polygon, mu agrees with the crossing-rule
    winding number."""
    verts = synth.star_polygon(24, 0.2, 0.45, seed=2)
    pts = synth.sample_polygon(verts, 8000).astype(np.float64)
    rng = np.random.default_rng(3)
    X = rng.random((400, 2))
    dist = oracle.polygon_distance(X, pts)
    X = X[dist > 0.05]
    mu = oracle.winding_number(X, pts)
    w = oracle.polygon_winding_exact(X, pts)
    # eq. kappdiscreteZ is a one-point rule per segment: error ~ spacing/distance
    np.testing.assert_allclose(mu, w, atol=2e-3)


def test_polygon_winding_exact_against_polar_test():
    """Crossing-rule winding number against an independent inside test for a
    star-shaped polygon: X is inside iff |X - c| is less than the radius of
    the edge crossed by the ray from c through X."""
    c = np.array([0.5, 0.5])
    verts = synth.star_polygon(24, 0.2, 0.45, seed=21)
    rng = np.random.default_rng(4)
    X = rng.random((2000, 2))
    w = oracle.polygon_winding_exact(X, verts)
    ang = np.mod(np.arctan2(X[:, 1] - c[1], X[:, 0] - c[0]), 2 * np.pi)
    j = np.floor(ang / (2 * np.pi / 24)).astype(int) % 24
    a, b = verts[j] - c, verts[(j + 1) % 24] - c
    u = (X - c) / np.linalg.norm(X - c, axis=1, keepdims=True)
    # ray t*u meets segment a + s (b - a): solve t u - s (b-a) = a
    den = u[:, 0] * -(b - a)[:, 1] - u[:, 1] * -(b - a)[:, 0]
    t = (a[:, 0] * -(b - a)[:, 1] - a[:, 1] * -(b - a)[:, 0]) / den
    inside = np.linalg.norm(X - c, axis=1) < t
    assert np.array_equal(w == 1, inside)
    assert set(np.unique(w)) <= {0, 1}


def test_polygon_distance_square():
    sq = np.array([[0.2, 0.2], [0.8, 0.2], [0.8, 0.8], [0.2, 0.8]])
    X = np.array([[0.5, 0.5], [0.1, 0.5], [0.9, 0.9], [0.5, 0.25]])
    np.testing.assert_allclose(oracle.polygon_distance(X, sq), [0.3, 0.1, np.sqrt(0.02), 0.05], atol=1e-15)


def test_degree_sphere_closed_form():
    """Sources on a sphere of radius rho about X with radial area vectors:
    every term of eq. normflux is |P_k|/rho^2, so mu = sum|P_k|/(4 pi rho^2)."""
    rng = np.random.default_rng(5)
    X = np.array([[0.4, 0.5, 0.6]])
    u = rng.standard_normal((300, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    rho = 0.17
    area = rng.random(300) * 1e-3
    Y = X + rho * u
    P = area[:, None] * u
    mu = oracle.topological_degree(X, Y, P)[0]
    assert mu == pytest.approx(area.sum() / (4 * np.pi * rho ** 2), rel=1e-13)
    # inward normals flip the sign
    assert oracle.topological_degree(X, Y, -P)[0] == pytest.approx(-mu, rel=1e-13)


def test_mesh_sources_incenter_and_area():
    """Incenter: equidistant from the three edge lines and inside the
    triangle; area vector: Heron's area along the right-hand normal."""
    rng = np.random.default_rng(6)
    V = rng.random((30, 3)).astype(np.float32)
    F = np.stack([np.arange(0, 30, 3), np.arange(1, 30, 3), np.arange(2, 30, 3)], axis=1).astype(np.int32)
    inc, P = oracle.mesh_sources(V, F)
    V64 = V.astype(np.float64)
    for k, (i, j, l) in enumerate(F):
        a, b, c = V64[i], V64[j], V64[l]

        def line_dist(p, u, v):
            w = v - u
            return np.linalg.norm(np.cross(p - u, w)) / np.linalg.norm(w)

        d = [line_dist(inc[k], a, b), line_dist(inc[k], b, c), line_dist(inc[k], c, a)]
        np.testing.assert_allclose(d, d[0], rtol=1e-10)
        la, lb, lc = np.linalg.norm(b - c), np.linalg.norm(c - a), np.linalg.norm(a - b)
        s = 0.5 * (la + lb + lc)
        heron = np.sqrt(s * (s - la) * (s - lb) * (s - lc))
        assert np.linalg.norm(P[k]) == pytest.approx(heron, rel=1e-9)
        n = np.cross(b - a, c - a)
        assert np.dot(P[k], n) > 0
        # inside: barycentric coordinates (a, b, c)/(a + b + c) are positive
        np.testing.assert_allclose(inc[k], (la * a + lb * b + lc * c) / (la + lb + lc), rtol=1e-12)


def test_degree_of_refined_sphere_mesh():
    """The degree of a closed outward mesh is close to 1 inside and 0 outside;
    the solid-angle winding number is exactly 1 / 0."""
    V, F = synth.generators.sphere_mesh(120, 80, 0.3, (0.5, 0.5, 0.5))
    inc, P = oracle.mesh_sources(V, F)
    X = np.array([[0.5, 0.5, 0.5], [0.6, 0.45, 0.52], [0.95, 0.5, 0.5], [0.1, 0.9, 0.2]])
    mu = oracle.topological_degree(X, inc, P)
    np.testing.assert_allclose(mu, [1, 1, 0, 0], atol=2e-3)
    np.testing.assert_allclose(oracle.mesh_winding_exact(X, V, F), [1, 1, 0, 0], atol=1e-9)


def test_mesh_winding_exact_cube():
    V, F = synth.cube_mesh(0.3, 0.7, subdiv=3)
    rng = np.random.default_rng(7)
    X = rng.random((500, 3))
    w = oracle.mesh_winding_exact(X, V, F)
    inside = np.all((X > 0.3) & (X < 0.7), axis=1)
    np.testing.assert_allclose(w, inside.astype(float), atol=1e-9)


def test_mesh_distance_cube():
    """Distance to the surface of a box against the closed form."""
    V, F = synth.cube_mesh(0.3, 0.7, subdiv=2)
    rng = np.random.default_rng(8)
    X = rng.random((200, 3))
    lo, hi = 0.3, 0.7
    inside = np.all((X > lo) & (X < hi), axis=1)
    d_in = np.minimum(X - lo, hi - X).min(axis=1)
    q = np.clip(X, lo, hi)
    d_out = np.linalg.norm(X - q, axis=1)
    expect = np.where(inside, d_in, d_out)
    np.testing.assert_allclose(oracle.mesh_distance(X, V, F), expect, atol=1e-7)


def test_label_rule():
    assert oracle.label_from_mu(np.array([0.0, 0.49, 0.5, 1.0, -1.0])).tolist() == [-1, -1, 1, 1, -1]
