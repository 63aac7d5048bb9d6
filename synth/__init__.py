"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This package holds grid recipes, method options and seeded random draws only.
It contains none of the method's arithmetic (no GLL points, no operators, no
solvers), so both sides can import it without sharing any computation.
"""
from .workloads import (  # noqa: F401
    Grid,
    Method,
    Workload,
    uniform_grid,
    geometric_spacing,
    random_spacing,
    c1_poisson2d_p4,
    c2_poisson3d_p8,
    c3_ldg3d_stretched,
    c4_batched,
    c5_poisson3d_p32,
    paper_periodic_2d,
    paper_fig6_2d,
    se_poisson3d_p8,
    rhs_uniform,
    guess_uniform01,
    with_method,
)
