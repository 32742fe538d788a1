"""Oracle-side helpers for the GPU parity tests.

Everything here is computed by the CPU oracle from the same seeded inputs
the GPU receives.  The padded sizes follow the library's documented rule
(next power of two >= 2n, at least 64), recomputed here and checked against
the plan.
"""

from __future__ import annotations

import os

import numpy as np

import oracle

# threads for the oracle's direct sums (the GPU hosts give one GPU 16 cores)
WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))

# Tolerances (absolute).  S: on every node against min(S_exact, S_max).
# Derivatives: on nodes with phi_exact >= 2 Theta ("deep valid").
TOL_S_TAU = 0.02            # |dS| <= 0.02 tau
TOL_GRAD = 0.02             # per component
TOL_HESS = 0.05             # times (1/tau + 1/h_min)
TOL_MU = 1e-3
TOL_S_TAU_FP64 = 1e-8       # float64 path, far above the validity threshold
TOL_GRAD_FP64 = 1e-8
# The float64 path's absolute error in phi is a few units of roundoff of the
# convolution; relative to phi it grows as Theta/phi.  The float64 bounds
# therefore allow TOL_THETA_FRAC * Theta/phi on top of the flat term: at the
# threshold that is the float32 tolerance, far above it the flat term rules.
TOL_THETA_FRAC = 0.02


def bound(ref, flat, scale=1.0):
    """Per-node absolute bound for the float64 path: scale*(flat + frac*Theta/phi)."""
    ratio = np.exp(np.log(ref["theta"]) - ref["lnphi"])
    return scale * (flat + TOL_THETA_FRAC * ratio)


def padded(n):
    m = 64
    while m < 2 * n:
        m *= 2
    return m


def padded_reduced(dims, spacing, tau, k_max, precision, c_theta=oracle.C_THETA):
    """Reduced padding of a single plan for calls with at most k_max sources:
    Theta_low = the threshold of one source on the full padding (a call with
    K sources has Theta >= sqrt(K) Theta_low); d_cut = tau (ln(c_theta
    sqrt(k_max)) - ln Theta_low); c_a = ceil(d_cut / h_a) cells; M_a = the
    smallest length >= max(64, n_a + c_a) among the powers of two, 288 and
    392, where that is below the full padding (else the full padding,
    untruncated).  Returns ((M_a...), (c_a...)) with c = 0 on a fully padded
    axis."""
    full = [padded(n) for n in dims]
    np_full = float(np.prod([float(m) for m in full]))
    u = 2.0 ** -53 if precision == "fp64" else 2.0 ** -24
    theta_low = c_theta * u * np.log2(np_full) / np.sqrt(np_full)
    d_cut = tau * (np.log(c_theta * np.sqrt(float(k_max))) - np.log(theta_low))
    Ms, cuts = [], []
    for n, h, Mf in zip(dims, spacing, full):
        c = int(np.ceil(d_cut / h))
        lengths = [1 << e for e in range(6, 13)] + [288, 392]
        Mr = min(m for m in lengths if m >= n + c)
        if Mr < Mf:
            Ms.append(Mr)
            cuts.append(c)
        else:
            Ms.append(Mf)
            cuts.append(0)
    return tuple(Ms), tuple(cuts)


def smooth7_at_least(n):
    """Smallest 2^a 3^b 5^c 7^d >= n."""
    m = max(int(n), 1)
    while True:
        r = m
        for p in (2, 3, 5, 7):
            while r % p == 0:
                r //= p
        if r == 1:
            return m
        m += 1


def batch_padded(n):
    """Padding rule of the batched path: M = 2 s, s the smallest 7-smooth >= n."""
    return 2 * smooth7_at_least(n)


def batch_padded_reduced(dims, spacing, tau, k_max, precision, c_theta=oracle.C_THETA):
    """Reduced padding rule of the batched path for calls with at most k_max
    sources: the validity threshold of one source on the full padding bounds
    every call's Theta from below, times sqrt(K) for K sources; d_cut = tau
    (ln(c_theta sqrt(k_max)) - ln Theta_low); c_a = ceil(d_cut / h_a) cells;
    M_a = 2 s, s the smallest 7-smooth >= (n_a + c_a) / 2, unless that is
    not below the full padding (then full padding and no truncation on that
    axis).  Returns
    ((M_x, M_y), (c_x, c_y)) with c = 0 on a fully padded axis."""
    full = [batch_padded(n) for n in dims]
    np_full = float(full[0]) * float(full[1])
    u = 2.0 ** -53 if precision == "fp64" else 2.0 ** -24
    theta_low = c_theta * u * np.log2(np_full) / np.sqrt(np_full)
    d_cut = tau * (np.log(c_theta * np.sqrt(float(k_max))) - np.log(theta_low))
    Ms, cuts = [], []
    for n, h, Mf in zip(dims, spacing, full):
        c = int(np.ceil(d_cut / h))
        Mr = 2 * smooth7_at_least((n + c + 1) // 2)
        if Mr < Mf:
            Ms.append(Mr)
            cuts.append(c)
        else:
            Ms.append(Mf)
            cuts.append(0)
    return tuple(Ms), tuple(cuts)


def reference(dims, spacing, origin, tau, pts, precision, *, grad=False, hess=False, cells=None,
              c_theta=oracle.C_THETA, padded_dims=None, rmean=False):
    """Oracle fields at all nodes (or at the given flat node indices)."""
    D = len(dims)
    idx, valid = oracle.snap(pts, origin, spacing, dims)
    Yh = oracle.node_coords(idx[valid], origin, spacing)
    _, mult = oracle.cell_multiplicities(idx[valid], dims)
    g_l2 = float(np.sqrt(np.sum(mult.astype(np.float64) ** 2)))
    Mp = tuple(padded(n) for n in dims) if padded_dims is None else tuple(padded_dims)
    l1 = oracle.kernel_l1(Mp, spacing, tau)
    theta = oracle.theta(precision, Mp, l1, g_l2, c_theta)
    smax = oracle.s_max(tau, theta)
    X = oracle.grid_nodes(dims, origin, spacing, cells)
    f = oracle.fields(X, Yh, tau, grad=grad, hess=hess, rmean=rmean, workers=WORKERS)
    lnphi = f["lnphi"]
    out = {
        "S_exact": f["S"],
        "lnphi": lnphi,
        "S_ref": np.minimum(f["S"], smax),
        "R": f["R"],
        "valid": lnphi >= np.log(theta),
        "deep": lnphi >= np.log(2 * theta),
        "theta": theta,
        "s_max": smax,
        "g_l2": g_l2,
        "padded": Mp,
        "kernel_l1": l1,
        "Yhat": Yh,
        "X": X,
    }
    if grad or hess:
        out["grad"] = f["grad"]
    if hess:
        out["hess"] = f["hess"]
    if rmean:
        out["rmean"] = f["rmean"]
    return out


def adjoint_noise(precision, padded_dims, l1, w_l2, c_theta=oracle.C_THETA):
    """Absolute rounding floor of the adjoint's FFT correlation at one source,
    by the same model as the validity threshold with the node weights w =
    G/phi in place of the source image: c_theta u log2(N_pad) ||f||_1
    ||w||_2 / sqrt(N_pad) (|u_i| <= f, so ||u_i||_1 <= ||f||_1)."""
    return oracle.theta(precision, padded_dims, l1, w_l2, c_theta)


# float64 adjoint: per component, the first-order effect of the forward's
# per-node error bound (relative error of phi e = TOL_S_TAU_FP64 +
# TOL_THETA_FRAC theta/phi, the bound the float64 S parity uses) on the node
# weights G/phi, plus the adjoint correlation's own rounding floor and
# float32 storage of dL/dY
STORE32 = 2.0 ** -23


def fp64_adjoint_bounds(sens_Y, sens_Y_theta, sens_tau, sens_tau_theta, noise, dY_ref):
    """Bounds on |dL/dY - ref| (K x D) and |dL/dtau - ref| from the
    sensitivities of oracle.l2_loss_gradients / source_weight_sums."""
    bY = (TOL_S_TAU_FP64 * sens_Y + TOL_THETA_FRAC * sens_Y_theta)[:, None] + noise + STORE32 * np.abs(dY_ref)
    bt = TOL_S_TAU_FP64 * sens_tau + TOL_THETA_FRAC * sens_tau_theta
    return bY, bt


def hess_components(H, D):
    """Stack an N x D x D Hessian in the library's channel order
    xx, xy, [xz,] yy, [yz,] zz."""
    pairs = [(0, 0), (0, 1), (1, 1)] if D == 2 else [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    return np.stack([H[:, i, j] for i, j in pairs], axis=0)
