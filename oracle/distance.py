"""Distance, gradient and Hessian by direct O(N K) sums in float64.

Definitions followed:

* R(X) = min_k ||X - Y_k||  (Sec. 1, eq. Rdef).
* phi(X) = sum_k exp(-||X - Y_k|| / tau)  (Sec. 2.3, eq. wavefunc) and
  S(X) = -tau log phi(X)  (Sec. 2.3, eq. STilde).  Evaluated as the
  equivalent log-sum-exp  S = R - tau log sum_k exp(-(r_k - R)/tau), which is
  identical in exact arithmetic and does not underflow for small tau.
* grad S = sum_k p_k n_k with p_k = exp(-r_k/tau)/phi and
  n_k = (X - Y_k)/r_k  (Sec. 5, eq. SxSy; written for x, the other axes
  follow "along similar lines").  At r_k = 0 the direction n_k is taken as 0
  (the paper sets the direction functions to 0 at the origin in Sec. 4.1).
* Hessian: H_ij = sum_k p_k [ -n_i n_j / tau + (delta_ij - n_i n_j)/r_k ]
  + S_i S_j / tau, summed over r_k > 0.  In 2D this is exactly eqs. Sxx, Syy
  and Sxy of Sec. 5 (with f_c = n_x, f_s = n_y, f_r = 1/r); the paper prints
  2D only, the D-dimensional form follows from the same differentiation of
  S = -tau log phi.
* <r> = sum_k p_k r_k  (used for dS/dtau = (S - <r>)/tau).
"""

from __future__ import annotations

import numpy as np

_CHUNK_ELEMS = 1 << 20   # node x source elements per chunk (sized for threads)


def _chunks(n_rows, k, per_elem=1):
    step = max(1, _CHUNK_ELEMS // max(1, k * per_elem))
    for s in range(0, n_rows, step):
        yield s, min(n_rows, s + step)


def run_chunks(fn, chunks, workers=1):
    """Apply fn(s, e) to every node chunk, on `workers` threads (NumPy
    releases the interpreter lock inside its array loops).  Each chunk writes
    only its own rows, so the result does not depend on the thread count;
    the return values come back in chunk order."""
    chunks = list(chunks)
    if workers <= 1 or len(chunks) <= 1:
        return [fn(s, e) for s, e in chunks]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(min(workers, len(chunks))) as ex:
        return list(ex.map(lambda c: fn(*c), chunks))


def nearest_distance(X, Y):
    """R(X) = min_k ||X - Y_k|| by brute force (Sec. 1, eq. Rdef)."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    out = np.empty(len(X))
    for s, e in _chunks(len(X), len(Y), X.shape[1]):
        d = X[s:e, None, :] - Y[None, :, :]
        out[s:e] = np.sqrt(np.einsum("ckd,ckd->ck", d, d)).min(axis=1)
    return out


def fields(X, Y, tau, grad=False, hess=False, rmean=False, workers=1):
    """Direct-sum fields at nodes X (N x D) from sources Y (K x D), float64.

    Returns a dict with ``R``, ``S``, ``lnphi`` (= log phi) and, on request,
    ``grad`` (N x D), ``hess`` (N x D x D) and ``rmean`` (N).  ``workers``
    threads share the node chunks (same values for any count).
    """
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    N, D = X.shape
    K = len(Y)
    if K == 0:
        raise ValueError("the distance field needs at least one source")
    tau = float(tau)
    out = {"R": np.empty(N), "S": np.empty(N), "lnphi": np.empty(N)}
    if grad or hess:
        out["grad"] = np.empty((N, D))
    if hess:
        out["hess"] = np.empty((N, D, D))
    if rmean:
        out["rmean"] = np.empty(N)
    eye = np.eye(D)
    per = D * D if hess else D

    def chunk(s, e):
        diff = X[s:e, None, :] - Y[None, :, :]               # X - Y_k
        r = np.sqrt(np.einsum("ckd,ckd->ck", diff, diff))
        R = r.min(axis=1)
        w = np.exp(-(r - R[:, None]) / tau)
        sw = w.sum(axis=1)
        out["R"][s:e] = R
        out["S"][s:e] = R - tau * np.log(sw)
        out["lnphi"][s:e] = -R / tau + np.log(sw)
        if grad or hess or rmean:
            p = w / sw[:, None]
        if rmean:
            out["rmean"][s:e] = np.einsum("ck,ck->c", p, r)
        if grad or hess:
            pos = r > 0
            inv_r = np.zeros_like(r)
            inv_r[pos] = 1.0 / r[pos]
            nvec = diff * inv_r[:, :, None]
            g = np.einsum("ck,ckd->cd", p, nvec)
            out["grad"][s:e] = g
            if hess:
                nn = nvec[:, :, :, None] * nvec[:, :, None, :]
                term = -nn / tau + (eye[None, None] - nn) * inv_r[:, :, None, None]
                # r_k = 0 terms: nvec = 0 and inv_r = 0, so -nn/tau = 0 and the
                # second term vanishes: they drop out as required.
                H = np.einsum("ck,ckij->cij", p, term) + g[:, :, None] * g[:, None, :] / tau
                out["hess"][s:e] = H

    run_chunks(chunk, _chunks(N, K, per), workers)
    return out


def distance_literal(X, Y, tau):
    """S = -tau log sum_k exp(-||X - Y_k||/tau) evaluated literally (no
    log-sum-exp shift), as printed in Sec. 2.3, eq. STilde."""
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    out = np.empty(len(X))
    for s, e in _chunks(len(X), len(Y), X.shape[1]):
        d = X[s:e, None, :] - Y[None, :, :]
        r = np.sqrt(np.einsum("ckd,ckd->ck", d, d))
        out[s:e] = -tau * np.log(np.exp(-r / tau).sum(axis=1))
    return out
