"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package draws meshes, coefficients and right-hand sides from fixed seeds.
It holds none of the smoother's arithmetic: no basis functions, no operators,
no transfers.  Both the oracle and the GPU library read the arrays it returns.
"""
from .generators import (  # noqa: F401
    Workload,
    WORKLOADS,
    workload,
    make_vertices,
    make_coefficients,
    make_rhs,
    make_case,
    make_random_patch,
    make_random_patches,
    make_sphere_distorted_patches,
    make_sphere_distorted_mesh,
    simplex_patch,
    make_simplex_patches,
)
