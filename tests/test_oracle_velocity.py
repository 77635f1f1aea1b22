"""Pin of the oracle's prescribed-velocity (VELO) right-hand side against the
pulsating sphere: uniform normal velocity u on a sphere of radius a radiates
p(a) = rho c u (i k a)/(i k a - 1) (time factor exp(-i w t); from the outgoing
monopole and Euler's equation).  The collocation solution converges to it at
first order in the element size: a wrong sign, a missing i k rho c factor or
a missing diagonal term of V would leave an O(1) error."""

import numpy as np

import synth
from oracle import velocity
from oracle.geometry import element_geometry
from oracle.presets import preset


def _err(level, k, rho_c=415.0, u0=1e-3):
    nodes, tris = synth.icosphere(level)
    g = element_geometry(nodes, tris)
    p = velocity.solve_velocity(g, k, np.full(len(tris), u0 + 0j), rho_c, p=preset("tight"))
    exact = rho_c * u0 * (1j * k) / (1j * k - 1.0)
    return np.max(np.abs(p - exact)) / abs(exact)


def test_pulsating_sphere_converges():
    e2, e3 = _err(2, 2.0), _err(3, 2.0)
    assert e3 < 0.03
    assert e3 < 0.65 * e2


def _cavity_err(level, k, rho_c=415.0, u0=1e-3):
    nodes, tris = synth.icosphere(level)
    g = element_geometry(nodes, tris)
    p = velocity.solve_velocity(g, k, np.full(len(tris), u0 + 0j), rho_c, p=preset("tight"), tau=-1)
    # inside a sphere of radius a (= 1) moving with normal velocity u: p = C sin(kr)/r,
    # dp/dr(a) = i k rho c u, so p(a) = rho c u i ka sin(ka) / (ka cos(ka) - sin(ka))
    exact = rho_c * u0 * 1j * k * np.sin(k) / (k * np.cos(k) - np.sin(k))
    return np.max(np.abs(p - exact)) / abs(exact)


def test_interior_cavity_converges():
    """tau = -1 (interior problem, Eq. (SystemI)): the field inside a pulsating
    spherical cavity; a wrong tau on the integral terms or on the jump term
    leaves an O(1) error."""
    e2, e3 = _cavity_err(2, 1.0), _cavity_err(3, 1.0)
    assert e3 < 0.04
    assert e3 < 0.65 * e2


def test_prescribed_pressure_recovers_pulsating_velocity():
    """PRES on the upper half of the sphere with the pulsating sphere's surface
    pressure and VELO with its velocity on the lower half: the solution holds
    dp/dn = i k rho c u on the PRES half and the analytic pressure on the VELO
    half (first-order discretisation error); swapping a PRES column for an A
    column or dropping the moved pressure term leaves an O(1) error."""
    nodes, tris = synth.icosphere(3)
    g = element_geometry(nodes, tris)
    N = len(tris)
    k, rho_c, u0 = 2.0, 415.0, 1e-3
    p_exact = rho_c * u0 * (1j * k) / (1j * k - 1.0)
    pres = np.nonzero(g["x"][:, 2] > 0.0)[0]
    velo = np.setdiff1d(np.arange(N), pres)
    u = np.zeros(N, dtype=np.complex128)
    u[velo] = u0
    pt = preset("tight")
    M, A0 = velocity.pressure_system(g, k, pres, p=pt)
    V = velocity.dense_dc(g, k, p=pt)
    rhs = velocity.pressure_rhs(A0, np.full(pres.size, p_exact)) - V[:, velo] @ (1j * k * rho_c * u[velo])
    x = np.linalg.solve(M, rhs)
    dpdn = 1j * k * rho_c * u0
    assert np.max(np.abs(x[pres] - dpdn)) / abs(dpdn) < 0.05
    assert np.max(np.abs(x[velo] - p_exact)) / abs(p_exact) < 0.05


def test_field_from_pressure_and_normal_derivative():
    """The representation formula with the surface pressure and its normal
    derivative given separately (oracle.field.field_pv), fed by the half-PRES,
    half-VELO solution above (p known on the PRES half, dp/dn the unknown
    there; p the unknown and dp/dn = i k rho c u on the VELO half): outside
    the sphere it must give the pulsating sphere's outgoing field
    p(r) = p(a) (a/r) exp(ik(r - a)).  Using c p in place of the prescribed
    derivative (zero here) or dropping the I^G term leaves an O(1) error."""
    from oracle import field
    nodes, tris = synth.icosphere(3)
    g = element_geometry(nodes, tris)
    N = len(tris)
    k, rho_c, u0 = 2.0, 415.0, 1e-3
    p_exact = rho_c * u0 * (1j * k) / (1j * k - 1.0)
    pres = np.nonzero(g["x"][:, 2] > 0.0)[0]
    velo = np.setdiff1d(np.arange(N), pres)
    u = np.zeros(N, dtype=np.complex128)
    u[velo] = u0
    pt = preset("tight")
    M, A0 = velocity.pressure_system(g, k, pres, p=pt)
    V = velocity.dense_dc(g, k, p=pt)
    rhs = velocity.pressure_rhs(A0, np.full(pres.size, p_exact)) - V[:, velo] @ (1j * k * rho_c * u[velo])
    x = np.linalg.solve(M, rhs)
    p_s = np.where(np.isin(np.arange(N), pres), p_exact, x)
    v_s = np.where(np.isin(np.arange(N), pres), x, 1j * k * rho_c * u0)
    pts = synth.points_on_sphere(12, 2.0, seed=3)
    f = field.field_pv(g, pts, k, p_s, v_s, p=pt)
    r = np.linalg.norm(pts, axis=1)
    exact = p_exact * np.exp(1j * k * (r - 1.0)) / r
    assert np.max(np.abs(f - exact)) / abs(exact[0]) < 0.03
    # the normal derivative matters: without it the field is far off
    f0 = field.field_pv(g, pts, k, p_s, np.zeros(N), p=pt)
    assert np.max(np.abs(f0 - exact)) / abs(exact[0]) > 0.3
