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
