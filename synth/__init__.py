"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds only input recipes: phantom shapes (disks, ellipses,
ellipsoids), the standard complex-normal draws used for noise, and the
workload parameter sets.  It contains none of the reconstruction method's
arithmetic (no Green's functions, no solves, no gradients, no proximal maps),
so that both the CPU oracle and the GPU path can take identical inputs from
it without sharing any of the computation that is being checked.
"""

from .phantoms import (  # noqa: F401
    disks_2d,
    mixed_2d,
    ellipses_2d,
    disk_area_fraction,
    ellipsoids_3d,
    complex_normal,
    random_field,
)
from .workloads import (  # noqa: F401
    BATCH_GRIDS,
    WORKLOADS,
    Workload,
    batched_uneven,
    fresnel3d_like_geometry,
    fresnel3d_like_sources,
    fresnel_like_geometry,
    two_spheres_3d,
    paper_sim_geometry,
)
