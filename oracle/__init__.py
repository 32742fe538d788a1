"""CPU FP64 oracle for the FFT distance-field path — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library
(``paper_1112_3010_amd``) never imports, links or calls it, and this package
never imports the product: the two share no code.  The only common module is
``synth`` (seeded input generators, which hold none of the method's
arithmetic).

What it computes, each by its plain definition in float64 with NumPy:

* ``discretize`` — snapping of sources to grid nodes (the paper places
  sources on grid nodes and rounds sampled inputs to them, Sec. 3 and 6).
* ``distance``   — R = min_k ||X - Y_k|| (Sec. 1, eq. Rdef);
  S = -tau log sum_k exp(-||X - Y_k||/tau) (Sec. 2.3, eq. STilde) written as a
  log-sum-exp; the gradient (Sec. 5, eq. SxSy) and the Hessian (Sec. 5,
  eqs. Sxx/Syy/Sxy, generalised to D dimensions) as weighted direct sums.
* ``sign``       — the discrete winding number (Sec. 4.1, eq. kappdiscreteZ)
  and topological degree (Sec. 4.2, eq. normflux) as direct sums, plus exact
  geometric inside/outside tests used to pin the labels.
* ``validity``   — the finite-precision validity threshold of the FFT path
  (a reading of Sec. 3.2, which the paper leaves qualitative).
* ``adjoint``    — gradients of a grid loss with respect to the sources and
  tau, by direct sums (derived from eq. STilde; not in the paper).
* ``table1``     — the paper's Table 1 algorithm (zero-padded FFT
  convolution) in float64 with ``numpy.fft``, for context timing and as an
  independent check of the grid conventions.
* ``metrics``    — the percentage error of Sec. 6.1 (eq. percentError).
* ``curvature``  — Gaussian, mean and principal curvatures from the gradient
  and Hessian (the derived quantities named at the end of Sec. 5): of the
  graph surface (x, y, S) in 2D, of the level surfaces of S in 3D.

Every function is pinned by ``tests/test_oracle_*.py`` against values that do
not come from the oracle itself (closed forms, the paper's bounds and printed
table, finite differences, brute force, library routines).
"""

from .discretize import snap, node_coords, grid_nodes, cell_multiplicities  # noqa: F401
from .distance import fields, distance_literal, nearest_distance  # noqa: F401
from .sign import (  # noqa: F401
    polygon_tangents,
    winding_number,
    mesh_sources,
    topological_degree,
    polygon_winding_exact,
    polygon_distance,
    mesh_winding_exact,
    mesh_distance,
    label_from_mu,
)
from .validity import kernel_l1, theta, s_max, UNIT_ROUNDOFF, C_THETA  # noqa: F401
from .adjoint import loss_gradients, l2_loss_gradients  # noqa: F401
from .metrics import percent_error  # noqa: F401
from .table1 import table1_distance, table1_phi  # noqa: F401
from .curvature import curvature, graph_curvature, level_set_curvature, G_MIN  # noqa: F401
