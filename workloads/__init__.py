"""Seeded synthetic inputs shared by the tests, the benchmark and the serving
demo: closed-form PEC cavity modes on the staggered grids and seeded problem
mixes.  This package holds no arithmetic of the scheme itself."""
from .cavity import (  # noqa: F401
    component_names, component_half_axes, field_shape, grid_coords,
    mode_fields, polarisation_3d, mode_omega,
)
from .mixes import batch_mix, serving_arrivals  # noqa: F401
