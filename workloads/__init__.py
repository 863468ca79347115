"""Seeded synthetic inputs for the 2D Stokes recursive-skeletonization path.

This package holds only input generation: boundary discretisations (nodes,
normals, trapezoid weights, curvature) of circles and ellipses, the random
multiply-connected geometries of the benchmark workloads, and boundary data
taken from exact Stokes flows (sums of point forces placed outside the fluid).
It contains none of the factorization's arithmetic and is shared, read-only,
by the CPU oracle and by the GPU library's tests and benchmark.
"""

from .geometry import (  # noqa: F401
    Curve,
    Geometry,
    ellipse_nodes,
    build_geometry,
    single_ellipse,
    concentric_annulus,
    random_holes_geometry,
    workload_small,
    workload_ellipse_2048,
    workload_circle10_8holes,
    workload_circle40_64holes,
    workload_batch_member,
    move_hole,
    insert_hole,
    delete_hole,
    starfish_nodes,
    starfish_geometry,
)
from .rhs import (  # noqa: F401
    PointForce,
    stokeslet_velocity,
    boundary_data,
    exterior_forces_for_geometry,
    neumann_flux,
)
