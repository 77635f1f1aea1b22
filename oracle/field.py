"""Exterior field points (oracle; test infrastructure only).

Eq. (BIE_I) with lambda = 1 at a point x outside the body and tau = 1:
    phi(x) = phi_inc(x) + sum_j ( int_Gj H(x, y) dy - c_j int_Gj G(x, y) dy ) phi_j,
with v_j = c_j phi_j.  The element integrals use the same quasi-singular and
regular rules as the collocation rows (Sec. 3.1.3-3.1.4), r~ measured from x.

With other boundary conditions (prescribed velocity, prescribed pressure)
the normal derivative is not c_j phi_j, and the same representation formula
takes the surface pressure and its normal derivative separately:
    phi(x) = phi_inc(x) + tau sum_j ( I^H_j(x) phi_j - I^G_j(x) v_j ),
with tau = -1 inside the fluid of an interior problem.

Pinned by: tests/test_oracle_operator.py (reciprocity of two point sources,
the analytic sphere field at r = 2); tests/test_oracle_velocity.py (the
pulsating sphere's outgoing field from a half-PRES, half-VELO solution);
tests/test_oracle_duct.py (the plane wave inside the duct of Sec. 5.3).
"""

import numpy as np

from .integrals import offdiag_integrals
from .operator import bc_factor


def field_parts(geom, pts, k, p=None):
    """(I^G, I^H), each of shape (n_pts, N): the element integrals of G and
    dG/dn_y seen from the field points."""
    pts = np.asarray(pts, dtype=np.float64)
    N = geom["x"].shape[0]
    IGm = np.zeros((pts.shape[0], N), dtype=np.complex128)
    IHm = np.zeros((pts.shape[0], N), dtype=np.complex128)
    dummy_n = np.tile(np.array([0.0, 0.0, 1.0]), (N, 1))
    for f in range(pts.shape[0]):
        xf = np.tile(pts[f], (N, 1))
        IG, IH, _, _ = offdiag_integrals(xf, dummy_n, geom["P0"], geom["P1"], geom["P2"],
                                         geom["n"], geom["A"], k, p)
        IGm[f] = IG
        IHm[f] = IH
    return IGm, IHm


def field_matrix(geom, pts, k, beta=None, p=None):
    """M with p_field = p_inc + M p_surface, shape (n_pts, N)."""
    IG, IH = field_parts(geom, pts, k, p)
    if beta is None:
        return IH
    return IH - bc_factor(k, beta)[None, :] * IG


def field_pv(geom, pts, k, p_surf, dpdn_surf, p=None, tau=1):
    """Scattered field tau sum_j (I^H_j p_j - I^G_j v_j) at the points, from
    the surface pressure p_surf and its normal derivative dpdn_surf (outward
    mesh normal); tau = -1 for points inside the fluid of an interior problem
    (Eq. (BIE_I) with the normals pointing out of the fluid)."""
    IG, IH = field_parts(geom, pts, k, p)
    return tau * (IH @ np.asarray(p_surf, dtype=np.complex128) - IG @ np.asarray(dpdn_surf, dtype=np.complex128))


def plane_wave(pts, k, d, P0=1.0):
    return P0 * np.exp(1j * k * (np.asarray(pts) @ np.asarray(d, dtype=np.float64)))


def point_source(pts, k, xs, P0=1.0):
    R = np.linalg.norm(np.asarray(pts) - np.asarray(xs), axis=1)
    return P0 * np.exp(1j * k * R) / (4.0 * np.pi * R)
