"""Curvatures derived from the distance field's first and second derivatives.

Test infrastructure (the oracle): plain float64 NumPy, called only by the
tests, the smoke check and the benchmark's CPU baseline.

Sec. 5 closes by noting that once S, its gradient and its Hessian are known on
the grid, the Gaussian, mean and principal curvatures of the two-dimensional
surface S(X) follow without further convolutions.  The paper gives no
formulas; the readings taken here:

* 2D grid: the surface is the graph (x, y, S(x, y)) (a Monge patch).  With
  W = 1 + S_x^2 + S_y^2:
    Gaussian  K = (S_xx S_yy - S_xy^2) / W^2
    mean      H = ((1 + S_y^2) S_xx - 2 S_x S_y S_xy + (1 + S_x^2) S_yy) / (2 W^(3/2))
  (the upward normal, so a surface opening upwards has H > 0).
* 3D grid: the surface is the level set of S through the node, with normal
  g / |g|, g = grad S.  With the Hessian H and its adjugate adj(H):
    mean      H_m = (|g|^2 tr H - g^T H g) / (2 |g|^3)
    Gaussian  K   = g^T adj(H) g / |g|^4
  (a sphere of radius rho around a single source has H_m = 1/rho,
  K = 1/rho^2).  Where |g| < g_min the level set is not defined by the
  derivatives; all four values are 0 there.
* principal curvatures k1 >= k2: H -/+ ... written k1,2 = H +/- sqrt(max(H^2 - K, 0)).
* Nodes outside the valid band carry zero derivatives; the formulas then give
  0 for every curvature (2D: W = 1, 3D: |g| = 0 < g_min).
"""

from __future__ import annotations

import numpy as np

# |grad S| below which the 3D level-set curvatures are reported as 0
G_MIN = 1e-3


def _principal(mean, gauss):
    s = np.sqrt(np.maximum(mean * mean - gauss, 0.0))
    return mean + s, mean - s


def graph_curvature(grad, hess):
    """Curvatures of the graph surface (x, y, S) from grad (N x 2) and the
    Hessian (N x 2 x 2).  Returns dict mean, gauss, k1, k2 (each N)."""
    g = np.asarray(grad, dtype=np.float64)
    h = np.asarray(hess, dtype=np.float64)
    sx, sy = g[:, 0], g[:, 1]
    hxx, hxy, hyy = h[:, 0, 0], h[:, 0, 1], h[:, 1, 1]
    W = 1.0 + sx * sx + sy * sy
    gauss = (hxx * hyy - hxy * hxy) / (W * W)
    mean = ((1.0 + sy * sy) * hxx - 2.0 * sx * sy * hxy + (1.0 + sx * sx) * hyy) / (2.0 * W ** 1.5)
    k1, k2 = _principal(mean, gauss)
    return {"mean": mean, "gauss": gauss, "k1": k1, "k2": k2}


def _adjugate_sym3(h):
    """Adjugate (transposed cofactor matrix) of symmetric 3 x 3 matrices."""
    a, b, c = h[:, 0, 0], h[:, 0, 1], h[:, 0, 2]
    d, e, f = h[:, 1, 1], h[:, 1, 2], h[:, 2, 2]
    adj = np.empty_like(h)
    adj[:, 0, 0] = d * f - e * e
    adj[:, 0, 1] = adj[:, 1, 0] = c * e - b * f
    adj[:, 0, 2] = adj[:, 2, 0] = b * e - c * d
    adj[:, 1, 1] = a * f - c * c
    adj[:, 1, 2] = adj[:, 2, 1] = b * c - a * e
    adj[:, 2, 2] = a * d - b * b
    return adj


def level_set_curvature(grad, hess, g_min=G_MIN):
    """Curvatures of the level surface of S through each node from grad
    (N x 3) and the Hessian (N x 3 x 3).  Returns dict mean, gauss, k1, k2."""
    g = np.asarray(grad, dtype=np.float64)
    h = np.asarray(hess, dtype=np.float64)
    q = np.einsum("ni,ni->n", g, g)
    ok = q >= g_min * g_min
    qs = np.where(ok, q, 1.0)
    tr = np.einsum("nii->n", h)
    gHg = np.einsum("ni,nij,nj->n", g, h, g)
    gAg = np.einsum("ni,nij,nj->n", g, _adjugate_sym3(h), g)
    mean = np.where(ok, (q * tr - gHg) / (2.0 * qs ** 1.5), 0.0)
    gauss = np.where(ok, gAg / (qs * qs), 0.0)
    k1, k2 = _principal(mean, gauss)
    return {"mean": mean, "gauss": gauss, "k1": np.where(ok, k1, 0.0), "k2": np.where(ok, k2, 0.0)}


def curvature(grad, hess, g_min=G_MIN):
    """Dispatch on the dimension of grad (2: graph surface, 3: level set)."""
    return graph_curvature(grad, hess) if np.asarray(grad).shape[1] == 2 else level_set_curvature(grad, hess, g_min)
