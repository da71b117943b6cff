"""Seeded synthetic workloads shared by the FP64 oracle and the HIP path.

This package only builds inputs (grids, bathymetry, Coriolis fields, initial
states, forcing snapshots).  It holds none of the finite-volume scheme's
arithmetic, so both implementations can consume the very same FP32 arrays.
The coastal generator builds its corner depths with a vectorised numpy
version of the bathymetry reconstruction of section "Bathymetry": part of
the input recipe, imported by neither the oracle nor the HIP library (the
device preprocessing is checked against the oracle on the raw cell depths
that ``coastal_cells`` returns).
"""

from .configs import (  # noqa: F401
    BC_NESTED,
    BC_PERIODIC,
    BC_WALL,
    FRIC_LINEAR,
    FRIC_MANNING,
    FRIC_NONE,
    FRIC_QUADRATIC,
    Workload,
    add_wind_field,
    coastal_cells,
    config1,
    config2,
    config3,
    config4_member,
    config4_sizes,
    config5_member,
    config5_requests,
    convergence_case,
    perimeter_len,
    random_small,
    rossby_case,
    rotate_ccw,
    unrotate_ccw,
)
