"""Seeded synthetic inputs (initial fields and random perturbations).

The one module that both the oracle-side tests and the GPU path draw inputs from.
It holds none of the method's arithmetic.
"""
from .fields import (  # noqa: F401
    isotropic_turbulence,
    random_fields,
    random_normal,
    taylor_green_2d,
    taylor_green_2d_on,
    taylor_green_3d,
    taylor_green_3d_on,
)
