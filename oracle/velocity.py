"""Prescribed normal velocity (VELO condition; oracle's own copy, test
infrastructure only).

Input appendix, boundary conditions: VELO fixes the normal particle velocity u
of an element; it may be combined with ADMI (a vibrating source on an
absorbing surface).  In Eq. (SystemI) the normal derivative of the pressure
unknown is then v = c phi + v_bar with v_bar = i w rho u = i k rho c u (time
factor exp(-i w t), normal pointing into the fluid), and the known part moves
to the right-hand side:

    A(c) phi = b - V v_bar,   V = dA/dc (G - gamma H' off the diagonal,
                                         G_ii - gamma/2 on it).

Pinned by tests/test_oracle_velocity.py against the pulsating sphere, whose
surface pressure is rho c u (i k a)/(i k a - 1) for a uniform u.
"""

import numpy as np

from .adjoint import dense_dc
from .operator import dense, lu_solve


def velocity_rhs(geom, k, u, rho_c, p=None, gamma=None, tau=1):
    """-V (i k rho c u): the right-hand-side term of prescribed velocities u."""
    V = dense_dc(geom, k, p=p, gamma=gamma, tau=tau)
    return -(V @ (1j * k * rho_c * np.asarray(u, dtype=np.complex128)))


def solve_velocity(geom, k, u, rho_c, beta=None, b=None, p=None, gamma=None, tau=1):
    """Pressure with prescribed velocities u (and admittance beta, incident b);
    tau = -1 for the interior problem."""
    rhs = velocity_rhs(geom, k, u, rho_c, p=p, gamma=gamma, tau=tau)
    if b is not None:
        rhs = rhs + b
    return lu_solve(dense(geom, k, beta, p, gamma, tau=tau), rhs)


def pressure_system(geom, k, pres, beta=None, p=None, gamma=None, tau=1):
    """System matrix with prescribed pressure (PRES) on the elements ``pres``
    (input appendix, boundary conditions): there the pressure is known and
    the unknown is v = dp/dn, so those columns of A are replaced by the
    columns of V = dA/dc; admittance on PRES elements is ignored."""
    pres = np.asarray(pres, dtype=np.int64)
    c_beta = None if beta is None else np.array(beta, dtype=np.complex128)
    if c_beta is not None:
        c_beta[pres] = 0.0
    M = dense(geom, k, c_beta, p, gamma, tau=tau)
    V = dense_dc(geom, k, p=p, gamma=gamma, tau=tau)
    A0_pres = M[:, pres].copy()  # the pressure columns (c = 0 there)
    M[:, pres] = V[:, pres]
    return M, A0_pres


def pressure_rhs(A0_pres, pres_values):
    """-A0[:, pres] p_bar: the known pressures moved to the right-hand side."""
    return -(A0_pres @ np.asarray(pres_values, dtype=np.complex128))
