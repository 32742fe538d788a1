"""The paper's Table 1 algorithm in float64 on the CPU (context only).

Steps (Sec. 3, Table 1): sample f(X) = exp(-||X||/tau) on the grid of
displacements; build g, the indicator of the source nodes (eqs. function_g,
krondelta, with multiplicity); transform both; multiply pointwise; invert;
take -tau log.  Reading: the paper does not mention padding, but the sum of
eq. wavefunc is a linear (not circular) convolution, so each axis is
zero-padded to M >= 2n - 1 (here the next power of two >= 2n).  Kernel
samples use the wrapped displacement d in [-M/2, M/2) with the d = -M/2
plane set to zero (never reached by an output node).
"""

from __future__ import annotations

import numpy as np


def _pad_len(n):
    m = 1
    while m < 2 * n:
        m *= 2
    return m


def table1_distance(idx, dims, spacing, tau, workers=None):
    """S on the full grid ([z][y][x]) from snapped source indices ``idx``
    (K x D ints), by zero-padded FFT convolution in float64."""
    phi = table1_phi(idx, dims, spacing, tau, workers=workers)
    with np.errstate(divide="ignore", invalid="ignore"):
        return -tau * np.log(phi)


def table1_phi(idx, dims, spacing, tau, dtype=np.float64, padded=None, workers=None):
    """phi on the full grid ([z][y][x]) by the zero-padded FFT convolution of
    Table 1, with every step (kernel samples, indicator, transforms, product,
    inverse) carried in ``dtype`` (float64 or float32; scipy's transforms keep
    single precision for float32 data).  ``padded`` gives the padded lengths
    (x first; default the next power of two >= 2n)."""
    dims = tuple(int(n) for n in dims)
    D = len(dims)
    Ms = tuple(_pad_len(n) for n in dims) if padded is None else tuple(int(m) for m in padded)
    # step 1: kernel on wrapped displacements, Nyquist planes zeroed
    grids = []
    for M, h in zip(Ms, spacing):
        d = np.arange(M, dtype=np.float64)
        d = np.where(d >= M // 2, d - M, d)
        grids.append(d * h)
    mesh = np.meshgrid(*grids[::-1], indexing="ij")       # (z, y, x) order
    r = np.sqrt(sum(m * m for m in mesh))
    f = np.exp(-r / tau)
    for ax in range(D):
        sl = [slice(None)] * D
        sl[ax] = Ms[::-1][ax] // 2
        f[tuple(sl)] = 0.0
    f = f.astype(dtype)
    # step 2: indicator (with multiplicity)
    g = np.zeros(Ms[::-1])
    np.add.at(g, tuple(np.asarray(idx)[:, ::-1].T), 1.0)
    g = g.astype(dtype)
    # steps 3-5
    import scipy.fft as sfft
    F = sfft.rfftn(f, workers=workers)
    Gs = sfft.rfftn(g, workers=workers)
    phi = sfft.irfftn(F * Gs, s=Ms[::-1], workers=workers)
    return phi[tuple(slice(0, n) for n in dims[::-1])]
