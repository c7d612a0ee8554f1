"""Seeded synthetic reservoir inputs shared by the CPU oracle tests and the GPU path.

This package only draws random fields and lays out configuration records
(grid sizes, fluid constants, well positions, step counts, solver settings).
It holds none of the method's arithmetic: no equation of state, no
transmissibility, no residual, no preconditioner.
"""
from .fields import gaussian_field, lognormal_perm, layered_perm, channel_perm  # noqa: F401
from .configs import (  # noqa: F401
    MD, DAY, ATM, Fluid, Problem, SolverSettings, Case,
    case_c1, case_c2, case_c3, case_c4, case_c5, small_case, with_solver,
)
