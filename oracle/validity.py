"""Finite-precision validity contract of the FFT path.

The paper notes (Sec. 3.2) that for small tau the FFT convolution in double
precision "tends to be erroneous" far from the sources, and escapes to
512-bit arithmetic.  It gives no quantitative rule.  Reading used by this
project (shared as a specification, not as code):

  An FFT convolution carries an absolute error of order
      phi_noise = u * log2(N_pad) * ||f||_1 * ||g||_2 / sqrt(N_pad)
  where u is the unit roundoff of the working precision, N_pad the number of
  points of the zero-padded grid, ||f||_1 the sum of the sampled kernel
  exp(-r/tau) over the padded grid (its Nyquist planes set to zero) and
  ||g||_2 = sqrt(sum over nodes of multiplicity^2).  A node is *valid* when
  phi >= Theta = C_THETA * phi_noise.  Invalid nodes report
  S_max = -tau log Theta and zero derivatives.

The reference value for parity is therefore min(S_exact, S_max).
"""

from __future__ import annotations

import math

import numpy as np

# "fp64x2": double-double (pairs of float64, 106 significand bits); its
# compound operations are accurate to a few units of 2^-106, taken as 2^-104.
# "fp64x4": quad-double (four float64 parts, 212 bits); its operations are
# accurate to a few units of 2^-211, taken as 2^-208.
UNIT_ROUNDOFF = {"fp32": 2.0 ** -24, "fp64": 2.0 ** -53, "fp64x2": 2.0 ** -104, "fp64x4": 2.0 ** -208}

#: Safety factor between the noise estimate and the validity threshold,
#: calibrated against the error of the Table 1 convolution carried out in
#: float32 (tests/test_oracle_adjoint.py): over every node of grids padded
#: to 64^2 ... 1024^2 and 64^3, 128^3 the largest |error of phi| is at most
#: 2.2 noise units, growing slowly with N_pad (the maximum of N roughly
#: Gaussian errors), so at phi = Theta the relative error is at most about
#: 2.2 / C_THETA and |dS| <= 0.02 tau holds up to 5 noise units.
C_THETA = 256.0


def kernel_l1(dims_pad, spacing, tau):
    """Sum of exp(-||h * d||/tau) over displacements d of the padded grid with
    -M_a/2 < d_a < M_a/2 on every axis (the Nyquist planes excluded)."""
    axes = []
    for M, h in zip(dims_pad, spacing):
        d = np.arange(0, M // 2, dtype=np.float64)     # d = 0 .. M/2 - 1
        w = np.where(d == 0, 1.0, 2.0)                  # +d and -d
        axes.append((d * h, w))
    if len(axes) == 2:
        (x, wx), (y, wy) = axes
        r = np.sqrt(x[None, :] ** 2 + y[:, None] ** 2)
        return float((np.exp(-r / tau) * wx[None, :] * wy[:, None]).sum())
    (x, wx), (y, wy), (z, wz) = axes
    total = 0.0
    for iz in range(len(z)):
        r = np.sqrt(x[None, :] ** 2 + y[:, None] ** 2 + z[iz] ** 2)
        total += wz[iz] * float((np.exp(-r / tau) * wx[None, :] * wy[:, None]).sum())
    return total


def theta(precision, dims_pad, l1, g_l2, c_theta=C_THETA):
    """Validity threshold Theta for the given working precision."""
    n_pad = float(np.prod(dims_pad))
    u = UNIT_ROUNDOFF[precision]
    return c_theta * u * math.log2(n_pad) * l1 * g_l2 / math.sqrt(n_pad)


def s_max(tau, theta_value):
    """S reported at invalid nodes: -tau log Theta."""
    return -tau * math.log(theta_value)
