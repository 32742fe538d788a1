"""Gradients of a grid loss with respect to the sources and tau.

Not in the paper; derived from its closed form S = -tau log sum_k
exp(-||X - Y_k||/tau) (Sec. 2.3, eq. STilde) by ordinary differentiation:

* dS(X)/dY_k = -p_k(X) n_k(X), with p_k = exp(-r_k/tau)/phi and
  n_k = (X - Y_k)/r_k (0 at r_k = 0, where the two one-sided derivatives of
  the cone cancel in a central difference).
* dS(X)/dtau = (S(X) - <r>(X)) / tau with <r> = sum_k p_k r_k.

For a loss L whose derivative with respect to the field is G = dL/dS, and a
validity mask (invalid nodes hold a constant, so they contribute nothing):
    dL/dY_k = -sum_{X valid} G(X) p_k(X) n_k(X)
    dL/dtau =  sum_{X valid} G(X) (S(X) - <r>(X)) / tau
"""

from __future__ import annotations

import numpy as np

_CHUNK_ELEMS = 1 << 21


def loss_gradients(X, Y, tau, G, mask=None):
    """Return (dL/dY as K x D float64, dL/dtau as float)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64).ravel()
    if mask is not None:
        keep = np.asarray(mask, dtype=bool).ravel() & (G != 0)
    else:
        keep = G != 0
    X = X[keep]
    G = G[keep]
    K, D = Y.shape
    dY = np.zeros((K, D))
    dtau = 0.0
    step = max(1, _CHUNK_ELEMS // max(1, K * D))
    for s in range(0, len(X), step):
        e = min(len(X), s + step)
        diff = X[s:e, None, :] - Y[None, :, :]
        r = np.sqrt(np.einsum("ckd,ckd->ck", diff, diff))
        R = r.min(axis=1)
        w = np.exp(-(r - R[:, None]) / tau)
        sw = w.sum(axis=1)
        p = w / sw[:, None]
        S = R - tau * np.log(sw)
        pos = r > 0
        inv_r = np.zeros_like(r)
        inv_r[pos] = 1.0 / r[pos]
        gp = G[s:e, None] * p                          # G(X) p_k(X)
        dY -= np.einsum("ck,ckd->kd", gp * inv_r, diff)
        rmean = np.einsum("ck,ck->c", p, r)
        dtau += float(np.dot(G[s:e], (S - rmean) / tau))
    return dY, dtau


def loss_value(X, Y, tau, G, mask=None):
    """L = sum_{X valid} G(X) S(X; Y, tau), the linear loss whose gradient
    :func:`loss_gradients` returns (used for finite-difference checks)."""
    from .distance import fields
    X = np.asarray(X, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64).ravel()
    keep = (G != 0) if mask is None else (np.asarray(mask, dtype=bool).ravel() & (G != 0))
    S = fields(X[keep], Y, tau)["S"]
    return float(np.dot(G[keep], S))
