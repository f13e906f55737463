"""Seeded synthetic workloads for the octree GIMP assembly.

This package only builds inputs: refinement criteria, material-point clouds placed on a
given set of octree leaves, material state, displacement and adjoint vectors. It holds
none of the method's arithmetic (no basis functions, no constitutive update, no octree
refinement); both the CPU oracle and the HIP library consume what it produces.
"""
from .configs import CONFIGS, Workload, get  # noqa: F401
from .generate import (  # noqa: F401
    PointSet, make_points, make_state, make_u, make_lambda, make_velocity, dirichlet_dofs, jitter_points,
)
