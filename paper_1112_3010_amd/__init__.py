"""MI355X (gfx950) fast-convolution signed distance fields.

Implements the method of Gurumoorthy and Rangarajan (arXiv:1112.3010):
S = -tau log sum_k exp(-||X - Y_k||/tau) on a regular grid by zero-padded
FFT convolution, its gradient and Hessian by further convolutions, the sign
by winding-number / topological-degree convolutions, and an adjoint for
gradients with respect to the sources and tau.  The compute path is the HIP
library libdt.so (C ABI in include/dt.h); this package is its binding.
"""

from ._lib import DtError, load as load_library  # noqa: F401
from .field import Plan, DistanceField, distance_field  # noqa: F401
from .batch import BatchPlan  # noqa: F401

__all__ = ["Plan", "BatchPlan", "DistanceField", "distance_field", "DtError", "load_library"]
