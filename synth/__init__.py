"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This package only *builds inputs*: triangle and quadrilateral meshes (vertex
coordinates and connectivity), random complex vectors, admittance arrays and field points.
It holds none of the boundary-element method's arithmetic (no element
geometry, no quadrature, no kernels), so both the CPU oracle and the HIP
library can be fed from it without sharing any of the method's code.
"""

from .meshes import (icosphere, geodesic_sphere, graded_ellipsoid_bump,
                     flat_patch, octahedron, box, box_quads, uv_sphere, mean_edge_length)
from .vectors import complex_normal, uniform01, points_on_sphere

__all__ = [
    "icosphere", "geodesic_sphere", "graded_ellipsoid_bump", "flat_patch",
    "octahedron", "box", "box_quads", "uv_sphere", "mean_edge_length", "complex_normal", "uniform01",
    "points_on_sphere",
]
