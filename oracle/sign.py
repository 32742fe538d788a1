"""Sign of the distance function: discrete winding number / topological degree
by direct sums, and exact geometric inside/outside tests.

Definitions followed:

* 2D (Sec. 4.1).  The closed curve is the ordered point list Y_1..Y_K with
  Y_{K+1} = Y_1; tangent Z_k = Y_{k+1} - Y_k (eq. tangentVec) and
  mu(X) = (1/2pi) sum_k [(Y_k^1 - X^1) Z_k^2 - (Y_k^2 - X^2) Z_k^1] / ||Y_k - X||^2
  (eq. kappdiscreteZ).  Terms with Y_k = X are dropped: the paper sets the
  direction kernels to 0 at the origin.  Reading: Y_k are the snapped
  sources, so mu is the winding number of the snapped closed polygon.
* 3D (Sec. 4.2).  Each triangle k contributes a centre Y_k (the incenter,
  which the paper offers as an example) and an outward normal P_k;
  mu(X) = (1/4pi) sum_k <Y_k - X, P_k> / ||Y_k - X||^3  (eq. normflux).
  Reading: P_k = (1/2)(v1 - v0) x (v2 - v0), the area vector, so that mu is
  close to 1 inside (the paper's unhalved cross product would give 2 and its
  threshold of 1 is then the same midpoint decision).
* Label (Sec. 6.1 and Example 5): +1 inside (mu >= 1/2), -1 outside.  The paper
  defines the signed distance as positive inside (Abstract, Sec. 4).
* Exact geometry (pins the labels, not part of the method): the crossing-rule
  winding number of the raw polygon and the solid-angle winding number of
  the raw mesh.
"""

from __future__ import annotations

import numpy as np

from .discretize import snap_f64

_CHUNK_ELEMS = 1 << 22


def _chunks(n_rows, k, per=1):
    step = max(1, _CHUNK_ELEMS // max(1, k * per))
    for s in range(0, n_rows, step):
        yield s, min(n_rows, s + step)


def polygon_tangents(Y):
    """Z_k = Y_{k+1} - Y_k with wrap-around (Sec. 4.1, eq. tangentVec)."""
    Y = np.asarray(Y, dtype=np.float64)
    return np.roll(Y, -1, axis=0) - Y


def winding_number(X, Y):
    """Discrete winding number of the closed polygon Y at nodes X
    (Sec. 4.1, eq. kappdiscreteZ), float64."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    Z = polygon_tangents(Y)
    out = np.empty(len(X))
    for s, e in _chunks(len(X), len(Y), 2):
        d = Y[None, :, :] - X[s:e, None, :]          # Y_k - X
        r2 = np.einsum("ckd,ckd->ck", d, d)
        num = d[:, :, 0] * Z[None, :, 1] - d[:, :, 1] * Z[None, :, 0]
        pos = r2 > 0
        q = np.zeros_like(r2)
        q[pos] = num[pos] / r2[pos]
        out[s:e] = q.sum(axis=1) / (2.0 * np.pi)
    return out


def mesh_sources(V, F):
    """Per-triangle incenter (float64, K x 3) and area vector
    P = (1/2)(v1 - v0) x (v2 - v0) (float64, K x 3) from float32 vertices.

    Evaluation order (fixed so that any implementation can reproduce the
    snapped node exactly): a = |v1 - v2|, b = |v2 - v0|, c = |v0 - v1| with
    |u| = sqrt((u_x*u_x + u_y*u_y) + u_z*u_z); incenter component
    = ((a*v0 + b*v1) + c*v2) / ((a + b) + c).
    """
    V = np.asarray(V, dtype=np.float32).astype(np.float64)
    F = np.asarray(F, dtype=np.int64)
    v0, v1, v2 = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]

    def norm(u):
        return np.sqrt((u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1]) + u[:, 2] * u[:, 2])

    a = norm(v1 - v2)
    b = norm(v2 - v0)
    c = norm(v0 - v1)
    den = (a + b) + c
    inc = ((a[:, None] * v0 + b[:, None] * v1) + c[:, None] * v2) / den[:, None]
    e1 = v1 - v0
    e2 = v2 - v0
    P = 0.5 * np.cross(e1, e2)
    return inc, P


def snapped_mesh_sources(V, F, origin, spacing, dims):
    """Incenters snapped to grid nodes (same rule as point sources), the
    node coordinates of the snapped centres, the area vectors, and the mask."""
    from .discretize import node_coords
    inc, P = mesh_sources(V, F)
    idx, valid = snap_f64(inc, origin, spacing, dims)
    return node_coords(idx, origin, spacing), P, idx, valid


def topological_degree(X, Y, P):
    """Normalised flux (1/4pi) sum_k <Y_k - X, P_k>/||Y_k - X||^3
    (Sec. 4.2, eq. normflux), float64; terms with Y_k = X dropped."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    P = np.asarray(P, dtype=np.float64)
    out = np.empty(len(X))
    for s, e in _chunks(len(X), len(Y), 3):
        d = Y[None, :, :] - X[s:e, None, :]
        r2 = np.einsum("ckd,ckd->ck", d, d)
        num = np.einsum("ckd,kd->ck", d, P)
        pos = r2 > 0
        q = np.zeros_like(r2)
        q[pos] = num[pos] / (r2[pos] * np.sqrt(r2[pos]))
        out[s:e] = q.sum(axis=1) / (4.0 * np.pi)
    return out


def label_from_mu(mu):
    """+1 where mu >= 1/2 (inside), -1 elsewhere (int8)."""
    return np.where(np.asarray(mu) >= 0.5, 1, -1).astype(np.int8)


# ---------------------------------------------------------------------------
# Exact geometry (pins for the labels)
# ---------------------------------------------------------------------------

def polygon_winding_exact(X, poly):
    """Integer winding number of the closed polygon ``poly`` (raw vertices,
    float64) about each X, by the crossing rule: an upward edge crossing with
    X strictly left of it adds 1, a downward crossing with X strictly right
    subtracts 1."""
    X = np.asarray(X, dtype=np.float64)
    a = np.asarray(poly, dtype=np.float64)
    b = np.roll(a, -1, axis=0)
    out = np.zeros(len(X), dtype=np.int64)
    for s, e in _chunks(len(X), len(a), 2):
        px = X[s:e, 0:1]
        py = X[s:e, 1:2]
        left = (b[None, :, 0] - a[None, :, 0]) * (py - a[None, :, 1]) - (px - a[None, :, 0]) * (
            b[None, :, 1] - a[None, :, 1])
        up = (a[None, :, 1] <= py) & (b[None, :, 1] > py) & (left > 0)
        down = (a[None, :, 1] > py) & (b[None, :, 1] <= py) & (left < 0)
        out[s:e] = up.sum(axis=1) - down.sum(axis=1)
    return out


def polygon_distance(X, poly):
    """Euclidean distance from each X to the closed polygon (its segments)."""
    X = np.asarray(X, dtype=np.float64)
    a = np.asarray(poly, dtype=np.float64)
    b = np.roll(a, -1, axis=0)
    ab = b - a
    L2 = np.einsum("kd,kd->k", ab, ab)
    out = np.empty(len(X))
    for s, e in _chunks(len(X), len(a), 2):
        ap = X[s:e, None, :] - a[None, :, :]
        t = np.einsum("ckd,kd->ck", ap, ab)
        t = np.where(L2[None, :] > 0, t / np.where(L2 > 0, L2, 1.0)[None, :], 0.0)
        t = np.clip(t, 0.0, 1.0)
        q = ap - t[:, :, None] * ab[None, :, :]
        out[s:e] = np.sqrt(np.einsum("ckd,ckd->ck", q, q)).min(axis=1)
    return out


def mesh_winding_exact(X, V, F):
    """Generalised winding number of a closed oriented triangle mesh about
    each X: the sum of signed solid angles over 4pi, each solid angle by the
    formula of Van Oosterom and Strackee (1983).  Equals 1 inside and 0
    outside for a closed, outward-wound surface."""
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float32).astype(np.float64)
    F = np.asarray(F, dtype=np.int64)
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    out = np.empty(len(X))
    for s, e in _chunks(len(X), len(F), 9):
        a = A[None] - X[s:e, None, :]
        b = B[None] - X[s:e, None, :]
        c = C[None] - X[s:e, None, :]
        la = np.sqrt(np.einsum("ckd,ckd->ck", a, a))
        lb = np.sqrt(np.einsum("ckd,ckd->ck", b, b))
        lc = np.sqrt(np.einsum("ckd,ckd->ck", c, c))
        det = np.einsum("ckd,ckd->ck", a, np.cross(b, c))
        den = (la * lb * lc + np.einsum("ckd,ckd->ck", a, b) * lc
               + np.einsum("ckd,ckd->ck", a, c) * lb + np.einsum("ckd,ckd->ck", b, c) * la)
        out[s:e] = (2.0 * np.arctan2(det, den)).sum(axis=1) / (4.0 * np.pi)
    return out


def _point_triangle_distance(p, a, b, c):
    """Distance from points p (M x 3) to triangles (a, b, c) (M x 3 each):
    the distance to the plane when the projection falls inside the triangle,
    else the least distance to the three edges."""
    def seg(p, u, v):
        uv = v - u
        L2 = np.einsum("md,md->m", uv, uv)
        t = np.einsum("md,md->m", p - u, uv) / np.where(L2 > 0, L2, 1.0)
        t = np.clip(t, 0.0, 1.0)
        q = u + t[:, None] * uv
        return np.sqrt(np.einsum("md,md->m", p - q, p - q))

    n = np.cross(b - a, c - a)
    nn = np.sqrt(np.einsum("md,md->m", n, n))
    nu = n / np.where(nn > 0, nn, 1.0)[:, None]
    dist_plane = np.einsum("md,md->m", p - a, nu)
    proj = p - dist_plane[:, None] * nu
    # inside test by edge-side signs relative to the normal
    s0 = np.einsum("md,md->m", np.cross(b - a, proj - a), n)
    s1 = np.einsum("md,md->m", np.cross(c - b, proj - b), n)
    s2 = np.einsum("md,md->m", np.cross(a - c, proj - c), n)
    inside = (s0 >= 0) & (s1 >= 0) & (s2 >= 0) & (nn > 0)
    edge = np.minimum(np.minimum(seg(p, a, b), seg(p, b, c)), seg(p, c, a))
    return np.where(inside, np.abs(dist_plane), edge)


def mesh_distance(X, V, F):
    """Exact Euclidean distance from each X to the triangle mesh.

    Candidate triangles for X are those with a vertex within d_v + e_max of X,
    where d_v is the distance to the nearest vertex and e_max the longest
    edge: every point of a triangle lies within its longest edge of each of
    its vertices, so the nearest triangle is always a candidate."""
    from scipy.spatial import cKDTree
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float32).astype(np.float64)
    F = np.asarray(F, dtype=np.int64)
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    e_max = max(np.linalg.norm(B - A, axis=1).max(), np.linalg.norm(C - B, axis=1).max(),
                np.linalg.norm(A - C, axis=1).max())
    # vertex -> incident triangles (CSR)
    order = np.argsort(F.ravel(), kind="stable")
    tri_of = order // 3
    counts = np.bincount(F.ravel(), minlength=len(V))
    start = np.concatenate([[0], np.cumsum(counts)])
    tree = cKDTree(V)
    dv, _ = tree.query(X, k=1)
    out = np.empty(len(X))
    for i, (x, d) in enumerate(zip(X, dv)):
        verts = tree.query_ball_point(x, d + e_max + 1e-12)
        tris = np.unique(np.concatenate([tri_of[start[v]:start[v + 1]] for v in verts]))
        p = np.broadcast_to(x, (len(tris), 3))
        out[i] = _point_triangle_distance(p, A[tris], B[tris], C[tris]).min()
    return out
