"""Seeded synthetic inputs (sparse PDE matrices and right-hand sides).

This package builds the linear systems A x = b that the solver and its
checker both consume.  It holds no part of the factorization itself: only
finite-difference matrix assembly, random coefficient fields and random
right-hand sides, all drawn from fixed seeds.
"""
from .pde import (  # noqa: F401
    CONFIGS,
    make_config,
    laplacian_2d,
    laplacian_3d,
    diffusion_2d,
    convection_diffusion_2d,
    helmholtz_2d,
    gaussian_random_field,
    random_rhs,
)
