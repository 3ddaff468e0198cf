"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and
the benchmark.

This package holds no arithmetic of the transport method itself.  It builds
what the method takes as input: boundary-conforming grids and their metric
G = J^{-1} J^{-T} in logical index units (Section 2.2, eq. (metric-eikonal)),
slowness models, source and receiver nodes, background traveltimes (analytic
fields of Section 5, or a first-arrival solve of eq. (eikonal)), and seeded
perturbation / data vectors.
"""
from .grids import (  # noqa: F401
    Workload,
    build,
    cell_velocities,
    config,
    curved_state,
    eikonal,
    eikonal_point,
    flat_radial,
    interpolating_receivers,
    manufactured,
    metric_from_coords,
    mu_g,
    perturbed_model,
    smooth_noise,
    small_3d,
    smooth_3d,
    traveltime_solver,
    data_noise,
    CONFIG_NAMES,
)
