"""Seeded synthetic lattice inputs shared by the GPU path and the oracle.

This module only draws random numbers and builds the input fields (gauge
links, sources, gauge transforms) in the canonical host layout.  It contains
none of the operator or solver arithmetic: both the oracle and the GPU library
take these arrays as inputs.
"""

from .fields import (  # noqa: F401
    GELL_MANN,
    canonical_shapes,
    site_coords,
    lattice_volume,
    rng_for,
    haar_su3,
    su3_exp_ieps_h,
    gauge_field,
    unit_gauge,
    gaussian_spinor,
    point_source,
    gauge_transform,
    SEEDS,
)
