"""Seeded synthetic inputs shared by the solver library's tests/benchmark and the oracle.

This package generates meshes and forcing data only; it contains none of the
discretisation or elimination arithmetic.
"""
from .mesh import cube_mesh, square_mesh  # noqa: F401
from .fields import (  # noqa: F401
    LinearisationField2D, Manufactured, constant_force, element_means, face_centroids,
    simplex_rule, element_points,
)
