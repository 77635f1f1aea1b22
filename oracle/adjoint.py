"""Gradient of a field-point objective with respect to element admittance
(oracle; test infrastructure only).

Objective: J(Y) = sum_f |p(x_f)|^2 over exterior field points, where the
surface pressure p solves the collocation system A(beta) p = b of
Eq. (SystemI) with beta_e = rho_c Y_e (Sec. 2.5; v = c p with
c = -i k beta), and p(x_f) follows from the representation formula,
Eq. (BIE_I) with lambda = 1.

The admittance enters A only through the factor c_j that multiplies column j
of the v-part, so A(c) = A0 + V diag(c) with
    V_ij = G_ij - gamma H'_ij  (i != j),     V_ii = G_ii - gamma/2,
and the field map is M(c) = I^H - I^G diag(c).  Differentiating
p_field = p_inc + M p with A p = b along Y_e (dc_e/dY_e = -i k rho_c):
    dJ/dY_e = 2 Re{ (dc_e/dY_e) p_e ( -conj((V^H mu)_e) - conj((I^G^H p_field)_e) ) },
    A^H mu = M^H p_field  (one adjoint solve).

Everything here is dense: V is assembled from its integrals directly, and
the solves are LAPACK LU.

Pinned by: tests/test_oracle_adjoint.py -- central finite differences of J
with the whole system re-assembled at each perturbed admittance, and
A(c) = A0 + V diag(c) against two independent dense assemblies.
"""

import numpy as np

from .field import field_parts
from .geometry import element_geometry
from .integrals import offdiag_integrals, self_integrals
from .operator import coupling, dense, lu_solve, rhs_plane_wave, rhs_point_source


def dense_dc(geom, k, p=None, gamma=None, tau=1):
    """V = dA/dc (the matrix that multiplies diag(c)), shape (N, N); tau = -1
    negates the integral terms of the interior problem (the -gamma/2 of the
    jump term stays)."""
    gamma = coupling(k, gamma, p)
    N = geom["x"].shape[0]
    V = np.zeros((N, N), dtype=np.complex128)
    ii, jj = np.nonzero(~np.eye(N, dtype=bool))
    block = 200000
    for s in range(0, ii.size, block):
        e = slice(s, s + block)
        IG, _, IHp, _ = offdiag_integrals(geom["x"][ii[e]], geom["n"][ii[e]], geom["P0"][jj[e]],
                                          geom["P1"][jj[e]], geom["P2"][jj[e]], geom["n"][jj[e]],
                                          geom["A"][jj[e]], k, p)
        V[ii[e], jj[e]] = tau * (IG - gamma * IHp)
    Gs, _ = self_integrals(geom, k, p)
    V[np.arange(N), np.arange(N)] = tau * Gs - 0.5 * gamma
    return V


def incident(pts, k, source):
    """Incident pressure at points; source = ("plane", d, P0) or ("point", x0, P0)."""
    kind, s, P0 = source
    pts = np.asarray(pts, dtype=np.float64)
    if kind == "plane":
        d = np.asarray(s, dtype=np.float64)
        d = d / np.linalg.norm(d)
        return P0 * np.exp(1j * k * (pts @ d))
    R = np.linalg.norm(pts - np.asarray(s, dtype=np.float64), axis=1)
    return P0 * np.exp(1j * k * R) / (4.0 * np.pi * R)


def _rhs(geom, k, source, p=None):
    kind, s, P0 = source
    if kind == "plane":
        d = np.asarray(s, dtype=np.float64)
        return rhs_plane_wave(geom, k, d / np.linalg.norm(d), P0, p=p)
    return rhs_point_source(geom, k, np.asarray(s, dtype=np.float64), P0, p=p)


def objective(nodes, tris, Y, k, rho_c, pts, source, p=None):
    """J and the intermediate fields, with the whole system assembled at Y."""
    geom = element_geometry(nodes, tris)
    beta = rho_c * np.asarray(Y, dtype=np.complex128)
    A = dense(geom, k, beta=beta, p=p)
    ps = lu_solve(A, _rhs(geom, k, source, p))
    IG, IH = field_parts(geom, pts, k, p)
    c = -1j * k * beta
    M = IH - IG * c[None, :]
    pf = incident(pts, k, source) + M @ ps
    return float(np.sum(np.abs(pf) ** 2)), {"geom": geom, "A": A, "p": ps, "IG": IG, "M": M, "pf": pf}


def gradient(nodes, tris, Y, k, rho_c, pts, source, p=None):
    """(J, dJ/dY) by one dense adjoint solve."""
    J, st = objective(nodes, tris, Y, k, rho_c, pts, source, p)
    V = dense_dc(st["geom"], k, p)
    mu = lu_solve(st["A"].conj().T, st["M"].conj().T @ st["pf"])
    w = V.conj().T @ mu
    hg = st["IG"].conj().T @ st["pf"]
    dc = -1j * k * rho_c
    g = 2.0 * np.real(dc * st["p"] * (-np.conj(w) - np.conj(hg)))
    return J, g, {"mu": mu, "w": w, "hg": hg, **st}
