"""Seeded synthetic media for the FLD radiation-energy update.

This package only draws random fields and lays out the workload recipes
(grid shapes, boundary conditions, densities, temperatures, time steps).
It holds none of the update's own arithmetic (no limiter, no face
coefficients, no solver, no exchange root), so the CPU oracle and the
GPU path can both consume its output without sharing any method code.
"""
from .generators import (  # noqa: F401
    grf,
    Medium,
    config_c1,
    config_c2,
    config_c3,
    config_c4,
    config_c5_train,
    config_amr,
    random_small_medium,
    velocity_field,
    KRAMERS,
)
