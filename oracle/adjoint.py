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

import math

import numpy as np

from .distance import run_chunks

_CHUNK_ELEMS = 1 << 19   # node x source elements per chunk (sized for threads)


def _node_chunks(n, K, D):
    step = max(1, _CHUNK_ELEMS // max(1, K * D))
    return [(s, min(n, s + step)) for s in range(0, n, step)]


def _pair_terms(X, Y, tau):
    """Per node of X and source k: X - Y_k, r_k, p_k, and per node S, log phi,
    <r> (the log-sum-exp form of eq. STilde)."""
    diff = X[:, None, :] - Y[None, :, :]
    r = np.sqrt(np.einsum("ckd,ckd->ck", diff, diff))
    R = r.min(axis=1)
    w = np.exp(-(r - R[:, None]) / tau)
    sw = w.sum(axis=1)
    p = w / sw[:, None]
    S = R - tau * np.log(sw)
    lnphi = -R / tau + np.log(sw)
    rmean = np.einsum("ck,ck->c", p, r)
    pos = r > 0
    inv_r = np.zeros_like(r)
    inv_r[pos] = 1.0 / r[pos]
    return diff, r, p, inv_r, S, lnphi, rmean


def loss_gradients(X, Y, tau, G, mask=None, workers=1):
    """Return (dL/dY as K x D float64, dL/dtau as float).  ``workers``
    threads share the node chunks; the partial sums are added in chunk
    order, so the result does not depend on the thread count."""
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

    def chunk(s, e):
        diff, r, p, inv_r, S, _, rmean = _pair_terms(X[s:e], Y, tau)
        gp = G[s:e, None] * p                          # G(X) p_k(X)
        return -np.einsum("ck,ckd->kd", gp * inv_r, diff), float(np.dot(G[s:e], (S - rmean) / tau))

    dY = np.zeros((K, D))
    dtau = 0.0
    for a, b in run_chunks(chunk, _node_chunks(len(X), K, D), workers):
        dY += a
        dtau += b
    return dY, dtau


def l2_loss_gradients(X, Y, tau, T, thetas, workers=1):
    """Gradients of L = sum over valid nodes of (S(X) - T(X))^2 at once for
    several validity thresholds, in one pass over the source pairs.

    For threshold theta (nodes with phi >= theta are valid; S_max = -tau log
    theta) the upstream gradient is G = 2 (min(S, S_max) - T) on every node
    and the gradients are those of :func:`loss_gradients` with that G and
    mask.  Returned with them are first-order sensitivities: if phi at each
    node X carries a relative error e(X) (so S carries -tau e and a node's
    weight G/phi carries e), dL/dY_k moves by at most
        sum_valid |G| |e| p_k            (since |n_k| <= 1)
    and dL/dtau = sum G (S - <r>)/tau by at most
        sum_valid |G| |e| (1 + 2 <r>/tau)
    (S moves by tau |e|, and <r> = (r f * g)/phi by at most 2 <r> |e|).
    They are given for e = 1 ("sens_Y", "sens_tau") and for e = theta/phi
    ("sens_Y_theta", "sens_tau_theta").

    Returns (S, lnphi, per_theta) with S and log phi at every node and
    per_theta a list of dicts with keys dY, dtau, sens_Y, sens_tau,
    sens_Y_theta, sens_tau_theta, n_valid.
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64).ravel()
    N, D = X.shape
    K = len(Y)
    S_all = np.empty(N)
    lnphi_all = np.empty(N)
    lnth = [math.log(t) for t in thetas]
    smax = [-tau * v for v in lnth]

    def chunk(s, e):
        diff, r, p, inv_r, S, lnphi, rmean = _pair_terms(X[s:e], Y, tau)
        S_all[s:e] = S
        lnphi_all[s:e] = lnphi
        res = []
        for lt, sm in zip(lnth, smax):
            valid = lnphi >= lt
            G = np.where(valid, 2.0 * (np.minimum(S, sm) - T[s:e]), 0.0)
            gp = G[:, None] * p
            dY = -np.einsum("ck,ckd->kd", gp * inv_r, diff)
            dtau = float(np.dot(G, (S - rmean) / tau))
            aG = np.abs(G)
            ratio = np.where(valid, np.exp(lt - lnphi), 0.0)     # theta / phi on valid nodes
            tw = 1.0 + 2.0 * rmean / tau
            res.append((dY, dtau, aG @ p, float(aG @ tw), (aG * ratio) @ p, float((aG * ratio) @ tw),
                        int(valid.sum())))
        return res

    per = [dict(dY=np.zeros((K, D)), dtau=0.0, sens_Y=np.zeros(K), sens_tau=0.0, sens_Y_theta=np.zeros(K),
                sens_tau_theta=0.0, n_valid=0) for _ in thetas]
    for res in run_chunks(chunk, _node_chunks(N, K, D), workers):
        for acc, (dY, dtau, sY, st, sYt, stt, nv) in zip(per, res):
            acc["dY"] += dY
            acc["dtau"] += dtau
            acc["sens_Y"] += sY
            acc["sens_tau"] += st
            acc["sens_Y_theta"] += sYt
            acc["sens_tau_theta"] += stt
            acc["n_valid"] += nv
    return S_all, lnphi_all, per


def source_weight_sums(X, Y, tau, C, workers=1):
    """sum over nodes X of C(X, j) p_k(X), for every source k and column j
    of C (N x m): K x m.  With C = |G| e, for a relative error e(X) of phi,
    this bounds how far dL/dY_k moves (|n_k| <= 1; see l2_loss_gradients)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64).reshape(len(X), -1)
    K, D = Y.shape

    def chunk(s, e):
        p = _pair_terms(X[s:e], Y, tau)[2]
        return p.T @ C[s:e]

    out = np.zeros((K, C.shape[1]))
    for part in run_chunks(chunk, _node_chunks(len(X), K, D), workers):
        out += part
    return out


def loss_value(X, Y, tau, G, mask=None):
    """L = sum_{X valid} G(X) S(X; Y, tau), the linear loss whose gradient
    :func:`loss_gradients` returns (used for finite-difference checks)."""
    from .distance import fields
    X = np.asarray(X, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64).ravel()
    keep = (G != 0) if mask is None else (np.asarray(mask, dtype=bool).ravel() & (G != 0))
    S = fields(X[keep], Y, tau)["S"]
    return float(np.dot(G[keep], S))


def l2_loss_value(X, Y, tau, T, theta):
    """L = sum over nodes of (min(S, S_max) - T)^2 with S_max = -tau log theta
    (for finite-difference checks of :func:`l2_loss_gradients`): a node with
    phi < theta holds S_max, so it adds a constant and no gradient."""
    from .distance import fields
    f = fields(np.asarray(X, dtype=np.float64), Y, tau)
    sm = -tau * math.log(theta)
    return float(np.sum((np.minimum(f["S"], sm) - np.asarray(T, dtype=np.float64).ravel()) ** 2))
