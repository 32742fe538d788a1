"""Seeded generators for the five synthetic workloads and for small test cases.

Every generator returns plain NumPy arrays in float32 (coordinates) or int32
(triangle indices).  Coordinates are physical: the grid covers [0, 1]^D with
``n`` cell-centred nodes per axis and spacing ``h = 1/n``.  Point arrays are
K x D with columns (x, y[, z]).  Field arrays are C-ordered [z][y][x].
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


# ---------------------------------------------------------------------------
# Point sets
# ---------------------------------------------------------------------------

def grid_cells_2d(n: int, k: int, seed: int) -> np.ndarray:
    """K distinct cells of an n x n grid drawn without replacement; returns the
    cell centres (i + 1/2)/n as float32 (exact for power-of-two n)."""
    rng = _rng(seed)
    flat = rng.choice(n * n, size=k, replace=False)
    iy, ix = np.divmod(flat, n)
    pts = np.stack([(ix + 0.5) / n, (iy + 0.5) / n], axis=1)
    return pts.astype(np.float32)


def random_grid_points(dims, k: int, seed: int, distinct: bool = False,
                       lo=None, hi=None) -> np.ndarray:
    """K points at uniformly random cell centres of a grid with ``dims`` nodes
    per axis (x first).  ``lo``/``hi`` restrict the cell index range per axis."""
    rng = _rng(seed)
    dims = [int(d) for d in dims]
    lo = [0] * len(dims) if lo is None else list(lo)
    hi = dims if hi is None else list(hi)
    if distinct:
        sizes = [h - l for l, h in zip(lo, hi)]
        total = int(np.prod(sizes))
        flat = rng.choice(total, size=k, replace=False)
        idx = np.stack(np.unravel_index(flat, sizes[::-1])[::-1], axis=1)
    else:
        idx = np.stack([rng.integers(l, h, size=k) for l, h in zip(lo, hi)], axis=1)
    idx = idx + np.asarray(lo)
    pts = (idx + 0.5) / np.asarray(dims, dtype=np.float64)
    return pts.astype(np.float32)


def grid_node_subset(n_axis: int, lo: float, h: float, k: int, seed: int) -> np.ndarray:
    """K distinct nodes, drawn without replacement, of the square grid with
    nodes lo + i h (i < n_axis per axis); float32 coordinates (x, y), exact
    for power-of-two h and lo.  The point sets of the 2D accuracy experiments
    (Sec. 6.1): Example 1 uses n_axis = 129, lo = -0.125, h = 1/512, k = 5000;
    Example 2 n_axis = 257, h = 1/1024, k = 10000."""
    rng = _rng(seed)
    flat = rng.choice(n_axis * n_axis, size=k, replace=False)
    iy, ix = np.divmod(flat, n_axis)
    return np.stack([lo + ix * h, lo + iy * h], axis=1).astype(np.float32)


def uniform_points(d: int, k: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """K points uniform in [lo, hi)^d (float32)."""
    rng = _rng(seed)
    return (lo + (hi - lo) * rng.random((k, d))).astype(np.float32)


# ---------------------------------------------------------------------------
# Closed polygons (2D sign input)
# ---------------------------------------------------------------------------

def star_polygon(n_vertices: int, rmin: float, rmax: float, seed: int,
                 centre=(0.5, 0.5)) -> np.ndarray:
    """A star-shaped polygon: vertex j at angle 2*pi*j/n with radius U[rmin,rmax]
    about ``centre``.  Vertices are counter-clockwise (float64, n x 2)."""
    rng = _rng(seed)
    theta = 2.0 * np.pi * np.arange(n_vertices) / n_vertices
    rad = rng.uniform(rmin, rmax, size=n_vertices)
    return np.stack([centre[0] + rad * np.cos(theta),
                     centre[1] + rad * np.sin(theta)], axis=1)


def sample_polygon(vertices: np.ndarray, k: int) -> np.ndarray:
    """K samples equispaced by arclength along the closed polygon, starting at
    vertex 0 and following the vertex order (float32, K x 2)."""
    v = np.asarray(vertices, dtype=np.float64)
    nxt = np.roll(v, -1, axis=0)
    seg = np.linalg.norm(nxt - v, axis=1)
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    total = cum[-1]
    s = np.arange(k) * (total / k)
    j = np.clip(np.searchsorted(cum, s, side="right") - 1, 0, len(v) - 1)
    t = (s - cum[j]) / seg[j]
    pts = v[j] + t[:, None] * (nxt[j] - v[j])
    return pts.astype(np.float32)


def regular_polygon(k: int, radius: float, centre, phase: float = 0.0) -> np.ndarray:
    """K vertices of a regular polygon, counter-clockwise (float64)."""
    th = phase + 2.0 * np.pi * np.arange(k) / k
    return np.stack([centre[0] + radius * np.cos(th), centre[1] + radius * np.sin(th)], axis=1)


# ---------------------------------------------------------------------------
# Closed triangle meshes (3D sign input)
# ---------------------------------------------------------------------------

def latlong_mesh(n_lon: int, n_ring: int, radius_fn, centre) -> tuple[np.ndarray, np.ndarray]:
    """Closed lat-long triangulation of a star-shaped surface.

    Vertices: north pole, ``n_ring`` rings of ``n_lon`` vertices at polar angle
    pi*j/(n_ring+1), south pole.  Vertex position = centre + radius_fn(dir)*dir.
    Triangles: n_lon (north cap) + (n_ring-1)*2*n_lon (bands) + n_lon (south cap),
    wound counter-clockwise as seen from outside.  Returns (V float32 nv x 3,
    F int32 nf x 3).
    """
    c = np.asarray(centre, dtype=np.float64)
    theta = np.pi * np.arange(1, n_ring + 1) / (n_ring + 1)
    phi = 2.0 * np.pi * np.arange(n_lon) / n_lon
    th, ph = np.meshgrid(theta, phi, indexing="ij")
    dirs = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=-1).reshape(-1, 3)
    dirs = np.concatenate([[[0.0, 0.0, 1.0]], dirs, [[0.0, 0.0, -1.0]]], axis=0)
    rad = np.asarray(radius_fn(dirs), dtype=np.float64)
    V = c + rad[:, None] * dirs

    def ring(j, i):  # vertex index of ring j (0-based), longitude i (mod n_lon)
        return 1 + j * n_lon + (i % n_lon)

    north, south = 0, 1 + n_ring * n_lon
    tris = []
    i = np.arange(n_lon)
    tris.append(np.stack([np.full(n_lon, north), ring(0, i), ring(0, i + 1)], axis=1))
    for j in range(n_ring - 1):
        a, b = ring(j, i), ring(j, i + 1)
        cc, d = ring(j + 1, i + 1), ring(j + 1, i)
        tris.append(np.stack([a, d, cc], axis=1))
        tris.append(np.stack([a, cc, b], axis=1))
    last = n_ring - 1
    tris.append(np.stack([np.full(n_lon, south), ring(last, i + 1), ring(last, i)], axis=1))
    F = np.concatenate(tris, axis=0).astype(np.int32)
    return V.astype(np.float32), F


def _real_sph_harm(l: int, m: int, dirs: np.ndarray) -> np.ndarray:
    from scipy.special import sph_harm_y
    polar = np.arccos(np.clip(dirs[:, 2], -1.0, 1.0))
    azim = np.arctan2(dirs[:, 1], dirs[:, 0])
    y = sph_harm_y(l, abs(m), polar, azim)
    if m > 0:
        return math.sqrt(2.0) * y.real
    if m < 0:
        return math.sqrt(2.0) * y.imag
    return y.real


def harmonic_star_mesh(seed: int, n_lon: int = 200, n_ring: int = 150, lmax: int = 6,
                       amplitude: float = 0.1, max_radius: float = 0.4,
                       centre=(0.5, 0.5, 0.5)) -> tuple[np.ndarray, np.ndarray]:
    """Unit sphere perturbed by random real spherical harmonics of degree 1..lmax,
    rho = 1 + amplitude * p / max|p|, then scaled so max rho = ``max_radius``.
    With the defaults this is the 60 000-triangle 3D signed workload."""
    rng = _rng(seed)
    coeffs = [(l, m, rng.standard_normal()) for l in range(1, lmax + 1) for m in range(-l, l + 1)]

    def p_of(dirs):
        return sum(a * _real_sph_harm(l, m, dirs) for l, m, a in coeffs)

    # Normalise on the mesh's own vertex directions.
    probe_V, _ = latlong_mesh(n_lon, n_ring, lambda d: np.ones(len(d)), (0.0, 0.0, 0.0))
    probe = probe_V.astype(np.float64)
    probe /= np.linalg.norm(probe, axis=1, keepdims=True)
    pmax = np.abs(p_of(probe)).max()
    rho_max = (1.0 + amplitude * p_of(probe) / pmax).max()
    scale = max_radius / rho_max

    def radius_fn(dirs):
        return scale * (1.0 + amplitude * p_of(dirs) / pmax)

    return latlong_mesh(n_lon, n_ring, radius_fn, centre)


def sphere_mesh(n_lon: int, n_ring: int, radius: float, centre) -> tuple[np.ndarray, np.ndarray]:
    """Lat-long triangulated sphere."""
    return latlong_mesh(n_lon, n_ring, lambda d: np.full(len(d), radius), centre)


def cube_mesh(lo, hi, subdiv: int = 1) -> tuple[np.ndarray, np.ndarray]:
    """Axis-aligned box [lo, hi]^3 with each face split into subdiv x subdiv
    quads of two triangles, wound counter-clockwise as seen from outside."""
    lo = np.asarray(lo, dtype=np.float64) * np.ones(3)
    hi = np.asarray(hi, dtype=np.float64) * np.ones(3)
    verts, faces = [], []
    t = np.linspace(0.0, 1.0, subdiv + 1)
    for axis in range(3):
        for side in (0, 1):
            u_ax, v_ax = [a for a in range(3) if a != axis]
            base = len(verts)
            for a in t:
                for b in t:
                    p = np.empty(3)
                    p[axis] = hi[axis] if side else lo[axis]
                    p[u_ax] = lo[u_ax] + a * (hi[u_ax] - lo[u_ax])
                    p[v_ax] = lo[v_ax] + b * (hi[v_ax] - lo[v_ax])
                    verts.append(p)
            for ia in range(subdiv):
                for ib in range(subdiv):
                    q00 = base + ia * (subdiv + 1) + ib
                    q10 = q00 + (subdiv + 1)
                    q01 = q00 + 1
                    q11 = q10 + 1
                    faces.extend([(q00, q10, q11), (q00, q11, q01)])
    V = np.asarray(verts)
    F = np.asarray(faces, dtype=np.int32)
    # Orient every face outward (the box is convex, so compare with the centre).
    cen = 0.5 * (lo + hi)
    a, b, c = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    nrm = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", nrm, (a + b + c) / 3.0 - cen) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V.astype(np.float32), F


# ---------------------------------------------------------------------------
# Differentiation workload inputs
# ---------------------------------------------------------------------------

def jittered_sphere_points(k: int, radius: float, jitter: float, seed: int,
                           centre=(0.5, 0.5, 0.5)) -> np.ndarray:
    """K points: Gaussian-normalised directions, radius ``radius + N(0, jitter^2)``."""
    rng = _rng(seed)
    d = rng.standard_normal((k, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius + jitter * rng.standard_normal(k)
    return (np.asarray(centre) + r[:, None] * d).astype(np.float32)


def ellipsoid_target(n: int, seed: int, n_samples: int = 200_000,
                     axes_range=(0.2, 0.35), centre=(0.5, 0.5, 0.5), cells=None) -> np.ndarray:
    """Unsigned distance on the n^3 cell-centred grid of [0,1]^3 to a random
    ellipsoid (axes U[axes_range], random rotation), approximated by the
    nearest of ``n_samples`` surface samples.  Returns float32 [z][y][x], or
    the values at the given flat node indices (x fastest) when ``cells`` is set."""
    from scipy.spatial import cKDTree
    rng = _rng(seed)
    axes = rng.uniform(axes_range[0], axes_range[1], size=3)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    u = rng.standard_normal((n_samples, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    surf = np.asarray(centre) + (u * axes) @ q.T
    tree = cKDTree(surf)
    if cells is not None:
        cells = np.asarray(cells, dtype=np.int64)
        ijk = np.stack([cells % n, (cells // n) % n, cells // (n * n)], axis=1)
        dist, _ = tree.query((ijk + 0.5) / n, k=1, workers=-1)
        return dist.astype(np.float32)
    c = (np.arange(n) + 0.5) / n
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    X = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    dist, _ = tree.query(X, k=1, workers=-1)
    return dist.reshape(n, n, n).astype(np.float32)


# ---------------------------------------------------------------------------
# Batched workload
# ---------------------------------------------------------------------------

def batch_instances(n_inst: int, seed_base: int, nmin: int = 128, nmax: int = 1024,
                    kmin: int = 100, kmax: int = 20000):
    """Independent square 2D instances: n = round(exp(U[ln nmin, ln nmax])),
    K = round(exp(U[ln kmin, ln kmax])), points uniform in [0,1)^2.
    Instance t uses seed ``seed_base + t``.  Returns a list of (n, Y)."""
    out = []
    for t in range(n_inst):
        rng = _rng(seed_base + t)
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        k = int(round(math.exp(rng.uniform(math.log(kmin), math.log(kmax)))))
        y = rng.random((k, 2)).astype(np.float32)
        out.append((n, y))
    return out


# ---------------------------------------------------------------------------
# The five named workloads
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    dims: tuple            # nodes per axis, x first
    taus: tuple            # tau values in physical units
    points: Optional[np.ndarray] = None      # K x D float32
    polygon: Optional[np.ndarray] = None     # 2D sign input: same as points (closed)
    vertices: Optional[np.ndarray] = None    # 3D sign input
    faces: Optional[np.ndarray] = None
    target: Optional[np.ndarray] = None      # S_target for the differentiation loss
    extra: Optional[dict] = None

    @property
    def ndim(self):
        return len(self.dims)

    @property
    def spacing(self):
        return tuple(1.0 / d for d in self.dims)

    @property
    def origin(self):
        return tuple(0.0 for _ in self.dims)


def workload(name: str, with_target: bool = True) -> Workload:
    """Build one of the named workloads (seed = its number)."""
    if name == "c1_2d_128":
        n = 128
        pts = grid_cells_2d(n, 64, seed=1)
        return Workload(name, (n, n), (2.0 / n,), points=pts)
    if name == "c2_2d_1024_polygon":
        n = 1024
        verts = star_polygon(24, 0.2, 0.45, seed=2)
        pts = sample_polygon(verts, 8000)
        return Workload(name, (n, n), (0.5 / n, 2.0 / n, 8.0 / n), points=pts, polygon=pts,
                        extra={"star_vertices": verts})
    if name == "c3_3d_256_mesh":
        n = 256
        V, F = harmonic_star_mesh(seed=3)
        return Workload(name, (n, n, n), (1.0 / n,), vertices=V, faces=F)
    if name == "c4_batch_2d":
        inst = batch_instances(96, seed_base=4000)
        return Workload(name, (), (), extra={"instances": inst})
    if name == "c5_3d_128_grad":
        n = 128
        pts = jittered_sphere_points(4096, 0.3, 2.0 / n, seed=5)
        tgt = ellipsoid_target(n, seed=5005) if with_target else None
        return Workload(name, (n, n, n), (4.0 / n,), points=pts, target=tgt)
    raise KeyError(name)


WORKLOADS = ("c1_2d_128", "c2_2d_1024_polygon", "c3_3d_256_mesh", "c4_batch_2d", "c5_3d_128_grad")
