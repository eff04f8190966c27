"""Seeded synthetic inputs for the space-time Navier-Stokes Newton systems.

This package is the one module that both the FP64 CPU oracle and the HIP path
read their inputs from.  It builds the problem, not the solver: structured
quadrilateral/hexahedral mesh hierarchies, the Q2/P1disc degree-of-freedom
maps, the dG(k) Gauss-Radau time matrices, the Newton Jacobian of the slab
system assembled on every multigrid level, the grid-transfer matrices, the
cell colouring and the seeded right-hand sides.  It contains none of the
smoother, multigrid or Krylov arithmetic.
"""
from .radau import radau_right, lagrange_at_nodes, dg_time_matrices
from .mesh import StructuredMesh, coarsen_shape, hierarchy_shapes
from .problems import CONFIGS, build_problem, build_hierarchy, Problem, Level

__all__ = [
    "radau_right", "lagrange_at_nodes", "dg_time_matrices",
    "StructuredMesh", "coarsen_shape", "hierarchy_shapes",
    "CONFIGS", "build_problem", "build_hierarchy", "Problem", "Level",
]
