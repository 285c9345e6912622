"""Seeded synthetic inputs for the learnable multigrid V-cycle.

Meshes, P1 finite-element matrices, prolongations, Galerkin hierarchies,
right-hand sides and parameter vectors.  This package is shared, as data, by
the CPU oracle (tests only) and the GPU path; it contains none of the
V-cycle's arithmetic.
"""
from . import fem, hierarchy, configs  # noqa: F401
