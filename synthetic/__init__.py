"""Seeded synthetic reservoir inputs shared by the CPU oracle tests and the GPU path.

This package only draws random fields and lays out configuration records
(grid sizes, fluid constants, well positions, step counts, solver settings).
It holds none of the method's arithmetic: no equation of state, no
transmissibility, no residual, no preconditioner.
"""
from .fields import gaussian_field, lognormal_perm, layered_perm, channel_perm, hzone_mask  # noqa: F401
from .configs import (  # noqa: F401
    MD, DAY, ATM, Fluid, Problem, SolverSettings, Case,
    case_2d_32, case_2d_512, case_3d_128, case_batch64, case_3d_96_adjoint, case_2d_flood, case_2d_flood_512,
    case_2d_hzone, case_3d_layered_flood,
    small_case,
    with_solver,
)
