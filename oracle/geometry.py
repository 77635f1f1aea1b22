"""Flat-triangle geometry (oracle; test infrastructure only).

Constant elements on flat triangles (Sec. 2.2 "Discretization of the
Geometry"); the collocation node of an element is the mean of its vertex
coordinates (Sec. 2.3 "Collocation"); counter-clockwise vertex order gives
the outward normal (appendix "The Mesh").

Pinned by: tests/test_oracle_geometry.py (area of the icosphere approaches
4*pi, normals are unit and outward, centroid of a known triangle).
"""

import numpy as np


def element_geometry(nodes, tris):
    """Return dict with P0, P1, P2 (N,3), centroid x (N,3), unit normal n (N,3)
    and area A (N,) for every triangle."""
    nodes = np.asarray(nodes, dtype=np.float64)
    tris = np.asarray(tris)
    P0 = nodes[tris[:, 0]]
    P1 = nodes[tris[:, 1]]
    P2 = nodes[tris[:, 2]]
    cr = np.cross(P1 - P0, P2 - P0)
    nrm = np.linalg.norm(cr, axis=1)
    return {
        "P0": P0, "P1": P1, "P2": P2,
        "x": (P0 + P1 + P2) / 3.0,
        "n": cr / nrm[:, None],
        "A": 0.5 * nrm,
    }
