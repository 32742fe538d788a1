"""Pins for the oracle's loss gradients and the validity contract (CPU only)."""

import numpy as np
import pytest

import oracle
from oracle.adjoint import loss_value


@pytest.mark.parametrize("d", [2, 3])
def test_source_gradient_matches_finite_differences(d):
    """dL/dY_k against central differences of L = sum G S in the continuous
    source positions (float64; the step is small enough that the truncation
    error, of order step^2/r^2, stays below the tolerance)."""
    rng = np.random.default_rng(20 + d)
    Y = rng.random((12, d))
    X = rng.random((300, d))
    X = X[oracle.nearest_distance(X, Y) > 0.02]   # the cone is smooth away from sources
    G = rng.standard_normal(len(X))
    tau = 0.05
    dY, dtau = oracle.loss_gradients(X, Y, tau, G)
    step = 1e-6
    fd = np.empty_like(Y)
    for k in range(len(Y)):
        for j in range(d):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[k, j] += step
            Ym[k, j] -= step
            fd[k, j] = (loss_value(X, Yp, tau, G) - loss_value(X, Ym, tau, G)) / (2 * step)
    np.testing.assert_allclose(dY, fd, rtol=2e-6, atol=1e-7)
    fdt = (loss_value(X, Y, tau + step, G) - loss_value(X, Y, tau - step, G)) / (2 * step)
    assert dtau == pytest.approx(fdt, rel=1e-6)


def test_mask_drops_nodes():
    rng = np.random.default_rng(30)
    Y = rng.random((8, 2))
    X = rng.random((100, 2))
    G = rng.standard_normal(100)
    mask = rng.random(100) > 0.5
    a = oracle.loss_gradients(X, Y, 0.05, G, mask)
    b = oracle.loss_gradients(X[mask], Y, 0.05, G[mask])
    np.testing.assert_allclose(a[0], b[0], rtol=1e-14)
    assert a[1] == pytest.approx(b[1], rel=1e-14)


def test_tau_derivative_nonpositive_for_positive_G():
    """dS/dtau <= 0 at every node (S <= R <= <r>), so G >= 0 gives dL/dtau <= 0."""
    rng = np.random.default_rng(31)
    Y = rng.random((20, 3))
    X = rng.random((200, 3))
    _, dtau = oracle.loss_gradients(X, Y, 0.03, np.abs(rng.standard_normal(200)))
    assert dtau <= 0


def test_kernel_l1_against_unfolded_sum():
    """kernel_l1 folds the padded grid by symmetry; compare with a literal
    sum over every displacement of a small padded grid (Nyquist planes out)."""
    for dims_pad, h, tau in [((16, 12), (0.1, 0.07), 0.13), ((8, 10, 6), (0.2, 0.15, 0.1), 0.2)]:
        axes = [np.arange(-M // 2 + 1, M // 2) * hh for M, hh in zip(dims_pad, h)]
        mesh = np.meshgrid(*axes, indexing="ij")
        r = np.sqrt(sum(m * m for m in mesh))
        assert oracle.kernel_l1(dims_pad, h, tau) == pytest.approx(np.exp(-r / tau).sum(), rel=1e-13)


def test_theta_scaling():
    """Theta grows linearly with ||f||_1, ||g||_2 and the unit roundoff."""
    t32 = oracle.theta("fp32", (64, 64), 10.0, 5.0)
    t64 = oracle.theta("fp64", (64, 64), 10.0, 5.0)
    assert t32 / t64 == pytest.approx(2.0 ** 29)
    assert oracle.theta("fp32", (64, 64), 20.0, 5.0) == pytest.approx(2 * t32)
    assert oracle.s_max(0.1, np.exp(-7.0)) == pytest.approx(0.7)


def _l2_case(d, seed, n_src=10, n_nodes=250, tau=0.06):
    rng = np.random.default_rng(seed)
    Y = rng.random((n_src, d))
    X = rng.random((n_nodes, d))
    X = X[oracle.nearest_distance(X, Y) > 0.02]
    T = 0.1 + 0.2 * rng.random(len(X))
    return X, Y, T, tau


@pytest.mark.parametrize("d", [2, 3])
def test_l2_loss_gradients_match_finite_differences(d):
    """dL/dY and dL/dtau of L = sum (min(S, S_max) - T)^2 against central
    differences of that loss in the continuous source positions and tau,
    for a threshold that cuts the node set (some nodes are invalid)."""
    from oracle.adjoint import l2_loss_value
    X, Y, T, tau = _l2_case(d, 40 + d)
    lnphi = oracle.fields(X, Y, tau)["lnphi"]
    theta = float(np.exp(np.quantile(lnphi, 0.3)))
    # keep nodes clear of the threshold, where the loss has a kink
    X, T = X[np.abs(lnphi - np.log(theta)) > 0.05], T[np.abs(lnphi - np.log(theta)) > 0.05]
    S, ln2, per = oracle.l2_loss_gradients(X, Y, tau, T, [theta])
    assert 0 < per[0]["n_valid"] < len(X)
    step = 1e-6
    fd = np.empty_like(Y)
    for k in range(len(Y)):
        for j in range(d):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[k, j] += step
            Ym[k, j] -= step
            fd[k, j] = (l2_loss_value(X, Yp, tau, T, theta) - l2_loss_value(X, Ym, tau, T, theta)) / (2 * step)
    np.testing.assert_allclose(per[0]["dY"], fd, rtol=2e-6, atol=1e-7)
    # tau enters S_max too; hold the threshold's S_max fixed as the library does
    theta_p = np.exp(np.log(theta) * tau / (tau + step))
    theta_m = np.exp(np.log(theta) * tau / (tau - step))
    fdt = (l2_loss_value(X, Y, tau + step, T, theta_p) - l2_loss_value(X, Y, tau - step, T, theta_m)) / (2 * step)
    assert per[0]["dtau"] == pytest.approx(fdt, rel=1e-5)


def test_l2_loss_sensitivities_by_brute_force():
    """The sensitivity sums written out with plain loops on a tiny case:
    sum over valid nodes of |G| p_k, of |G| (theta/phi) p_k, and the tau
    weights (1 + 2 <r>/tau)."""
    X, Y, T, tau = _l2_case(2, 50, n_src=4, n_nodes=30, tau=0.08)
    lnphi = oracle.fields(X, Y, tau)["lnphi"]
    theta = float(np.exp(np.median(lnphi)))
    S, ln2, per = oracle.l2_loss_gradients(X, Y, tau, T, [theta, theta * 1e-6])
    for th, acc in zip([theta, theta * 1e-6], per):
        sY = [0.0] * len(Y)
        sYt = [0.0] * len(Y)
        st = stt = 0.0
        nv = 0
        for i, x in enumerate(X):
            r = [float(np.sqrt(((x - y) ** 2).sum())) for y in Y]
            e = [np.exp(-rk / tau) for rk in r]
            phi = sum(e)
            if phi < th:
                continue
            nv += 1
            s = -tau * np.log(phi)
            g = abs(2 * (min(s, -tau * np.log(th)) - T[i]))
            rm = sum(ek * rk for ek, rk in zip(e, r)) / phi
            for k in range(len(Y)):
                sY[k] += g * e[k] / phi
                sYt[k] += g * (th / phi) * e[k] / phi
            st += g * (1 + 2 * rm / tau)
            stt += g * (th / phi) * (1 + 2 * rm / tau)
        assert acc["n_valid"] == nv
        valid = oracle.fields(X, Y, tau)["lnphi"] >= np.log(th)
        G = np.where(valid, np.abs(2 * (np.minimum(S, -tau * np.log(th)) - T)), 0.0)
        C = np.stack([G, G * np.exp(np.log(th) - ln2)], axis=1)
        ws = oracle.adjoint.source_weight_sums(X, Y, tau, C)
        np.testing.assert_allclose(ws[:, 0], sY, rtol=1e-12)
        np.testing.assert_allclose(ws[:, 1], sYt, rtol=1e-12)
        np.testing.assert_allclose(acc["sens_Y"], sY, rtol=1e-12)
        np.testing.assert_allclose(acc["sens_Y_theta"], sYt, rtol=1e-12)
        assert acc["sens_tau"] == pytest.approx(st, rel=1e-12)
        assert acc["sens_tau_theta"] == pytest.approx(stt, rel=1e-12)


def test_worker_threads_do_not_change_results():
    X, Y, T, tau = _l2_case(3, 60, n_src=1000, n_nodes=3000)   # several node chunks
    G = np.random.default_rng(61).standard_normal(len(X))
    a = oracle.loss_gradients(X, Y, tau, G, workers=1)
    b = oracle.loss_gradients(X, Y, tau, G, workers=4)
    assert np.array_equal(a[0], b[0]) and a[1] == b[1]
    f1 = oracle.fields(X, Y, tau, grad=True, hess=True, workers=1)
    f4 = oracle.fields(X, Y, tau, grad=True, hess=True, workers=4)
    for key in f1:
        assert np.array_equal(f1[key], f4[key]), key


def _fft32_error(dims, K, tau_cells, seed):
    """Absolute error of phi from the Table 1 convolution carried out in
    float32 (scipy.fft) against the direct sum, with the padding of the
    library's rule, and the validity threshold's noise model for that case."""
    rng = np.random.default_rng(seed)
    D = len(dims)
    h = tuple(1.0 / dims[0] for _ in dims)
    tau = tau_cells * h[0]
    idx = np.stack([rng.integers(0, n, K) for n in dims], axis=1)
    Mp = tuple(max(64, 1 << int(np.ceil(np.log2(2 * n)))) for n in dims)
    phi32 = oracle.table1_phi(idx, dims, h, tau, dtype=np.float32, padded=Mp).astype(np.float64).ravel()
    f = oracle.fields(oracle.grid_nodes(dims, (0.0,) * D, h), oracle.node_coords(idx, (0.0,) * D, h), tau, workers=4)
    _, mult = oracle.cell_multiplicities(idx, dims)
    g_l2 = float(np.sqrt(np.sum(mult.astype(np.float64) ** 2)))
    theta = oracle.theta("fp32", Mp, oracle.kernel_l1(Mp, h, tau), g_l2)
    err = np.abs(phi32 - np.exp(f["lnphi"]))
    with np.errstate(divide="ignore", invalid="ignore"):
        dS = np.abs(-tau * np.log(phi32) - f["S"])
    return float(np.prod(Mp)), err, theta / oracle.C_THETA, theta, np.exp(f["lnphi"]), dS, tau


def test_theta_noise_model_against_float32_fft():
    """The form of the validity threshold, pinned outside the library: the
    Table 1 convolution in float32 (scipy's transforms) at padded sizes from
    64^2 to 512^2 and 64^3 to 128^3.  (i) The rms error of phi over the grid
    is the same fraction of the noise model u log2(N_pad) ||f||_1 ||g||_2 /
    sqrt(N_pad) at every size (within [0.01, 0.5], and without a trend in
    N_pad: a wrong power of N_pad would change it by the size ratio);
    (ii) |dS| <= 0.02 tau on every node with phi >= Theta, the contract's
    tolerance, and the largest error stays below c_theta * 0.02 noise units;
    (iii) near the threshold (Theta <= phi < 4 Theta) the error is not
    negligible: at least 1/2000 of the tolerance, so the threshold is not
    placed far inside the region where float32 is exact."""
    cases = [((n, n), 200, 1.0, n + 1) for n in (32, 64, 128, 256)] + \
            [((n, n, n), 30, 1.5, n + 2) for n in (32, 48)]
    npad, rms = [], []
    for dims, K, tc, seed in cases:
        N_pad, err, noise, theta, phi, dS, tau = _fft32_error(dims, K, tc, seed)
        r = float(np.sqrt(np.mean(err ** 2)) / noise)
        assert 0.01 <= r <= 0.5, (dims, r)
        assert err.max() <= 0.02 * oracle.C_THETA * noise, dims
        valid = phi >= theta
        assert dS[valid].max() <= 0.02 * tau, dims
        near = valid & (phi < 4 * theta)
        if near.any():
            assert dS[near].max() >= 0.02 * tau / 2000, dims
        if len(dims) == 2:
            npad.append(N_pad)
            rms.append(r)
    slope = np.polyfit(np.log(npad), np.log(rms), 1)[0]
    assert abs(slope) < 0.25, slope
