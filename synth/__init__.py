"""Seeded synthetic inputs for the distance-field path.

This module only draws inputs (point sets, closed polygons, closed triangle
meshes, target fields).  It contains none of the method's arithmetic: no
snapping to the grid, no kernels, no convolutions, no triangle centres or
normals.  Both the CPU oracle and the GPU tests/bench take their inputs from
here, so that the two sides see identical data.

Seeding convention: workload ``c`` uses ``numpy.random.default_rng(c)``;
trial or instance ``t`` of workload ``c`` uses ``default_rng(1000 * c + t)``.
"""

from .generators import (  # noqa: F401
    Workload,
    grid_cells_2d,
    random_grid_points,
    star_polygon,
    sample_polygon,
    latlong_mesh,
    harmonic_star_mesh,
    cube_mesh,
    jittered_sphere_points,
    ellipsoid_target,
    batch_instances,
    workload,
    WORKLOADS,
)
