"""Placement of sources on the grid.

The method evaluates its sums only for sources that sit on grid nodes
(Sec. 1 and Sec. 3: the Kronecker-delta indicator g is defined on the grid);
every experiment rounds sampled input to grid nodes (Sec. 6, Examples 3-5).

Reading used here (the paper does not fix a rounding rule): the grid has
n_d cell-centred nodes per axis, node i at o_d + (i + 1/2) h_d.  A source
y (given in float32) belongs to node idx_d = floor((y_d - o_d) / h_d),
evaluated in float64 with IEEE division.  A point on a cell face therefore
goes to the upper cell.  A point with idx_d outside [0, n_d) is rejected.
Coincident sources count with multiplicity.
"""

from __future__ import annotations

import numpy as np


def snap(points, origin, spacing, dims):
    """Return (idx, valid): int64 K x D node indices and a K bool mask.

    ``points`` are converted to float32 first (the library takes float32
    input), then to float64, so both sides see identical values.
    """
    y = np.asarray(points, dtype=np.float32).astype(np.float64)
    o = np.asarray(origin, dtype=np.float64)
    h = np.asarray(spacing, dtype=np.float64)
    n = np.asarray(dims, dtype=np.int64)
    q = np.floor((y - o) / h)
    finite = np.all(np.isfinite(q), axis=1)
    q = np.where(np.isfinite(q), q, -1.0)
    idx = q.astype(np.int64)
    valid = finite & np.all((idx >= 0) & (idx < n), axis=1)
    return idx, valid


def snap_f64(points64, origin, spacing, dims):
    """Like :func:`snap` for coordinates that are already float64 (triangle
    centres computed in float64)."""
    y = np.asarray(points64, dtype=np.float64)
    o = np.asarray(origin, dtype=np.float64)
    h = np.asarray(spacing, dtype=np.float64)
    n = np.asarray(dims, dtype=np.int64)
    q = np.floor((y - o) / h)
    finite = np.all(np.isfinite(q), axis=1)
    q = np.where(np.isfinite(q), q, -1.0)
    idx = q.astype(np.int64)
    valid = finite & np.all((idx >= 0) & (idx < n), axis=1)
    return idx, valid


def node_coords(idx, origin, spacing):
    """Physical coordinates o + (idx + 1/2) h of integer node indices (float64)."""
    return np.asarray(origin, dtype=np.float64) + (np.asarray(idx, dtype=np.float64) + 0.5) * np.asarray(
        spacing, dtype=np.float64)


def grid_nodes(dims, origin, spacing, flat=None):
    """Node coordinates (N x D, float64) for all nodes in C order [z][y][x]
    (x fastest), or for the given flat indices into that order."""
    dims = tuple(int(d) for d in dims)
    total = int(np.prod(dims))
    flat = np.arange(total) if flat is None else np.asarray(flat, dtype=np.int64)
    unr = np.unravel_index(flat, dims[::-1])      # (z, y, x) or (y, x)
    idx = np.stack(unr[::-1], axis=1)             # columns x, y[, z]
    return node_coords(idx, origin, spacing)


def cell_multiplicities(idx, dims):
    """Return (unique node indices U x D, multiplicity per unique node)."""
    idx = np.asarray(idx, dtype=np.int64)
    if len(idx) == 0:
        return idx.reshape(0, len(dims)), np.zeros(0, dtype=np.int64)
    u, m = np.unique(idx, axis=0, return_counts=True)
    return u, m
