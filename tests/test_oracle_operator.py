"""Pins for the whole dense operator: closed forms on the sphere and
reciprocity (discretisation-limited, so the checks are on the error level
and its decrease under refinement)."""

import numpy as np
import pytest
from scipy.special import eval_legendre

import synth
from oracle import operator as op
from oracle import sphere, field
from oracle.geometry import element_geometry
from oracle.presets import preset


def _modal_err(subdiv, k, n, beta=0.0, gamma=None):
    nodes, tris = synth.icosphere(subdiv)
    g = element_geometry(nodes, tris)
    A = op.dense(g, k, beta=None if beta == 0 else np.full(len(tris), beta), p=preset("paper"),
                 gamma=gamma)
    ct = g["x"][:, 2] / np.linalg.norm(g["x"], axis=1)
    f = eval_legendre(n, ct)
    lam = sphere.bm_eigenvalue(n, k, beta=beta, gamma=gamma)
    return np.linalg.norm(A @ f - lam * f) / np.linalg.norm(lam * f)


@pytest.mark.parametrize("n", [0, 1, 3, 5])
def test_double_layer_modal_eigenvalues_converge(n):
    # gamma = 0 leaves 1/2 - K: the collocated double layer converges for
    # every degree (second order on the icosphere)
    k = 2.0
    e2 = _modal_err(2, k, n, gamma=0.0)
    e3 = _modal_err(3, k, n, gamma=0.0)
    assert e3 < 0.6 * e2 and e3 < 0.1


@pytest.mark.parametrize("n", [0, 1])
def test_modal_eigenvalues_converge(n):
    # With the hypersingular part the centroid-collocated constant-element
    # error stalls at a few per cent for higher degrees (the piecewise-constant
    # interpolation error is not smoothed by an order-one operator), so the
    # full Burton-Miller operator is checked on the low degrees.
    k = 2.0
    e2 = _modal_err(2, k, n)
    e3 = _modal_err(3, k, n)
    assert e3 < 0.05
    assert e3 < 0.6 * e2


def test_modal_eigenvalues_with_admittance():
    k, n, beta = 2.0, 0, 0.8 + 0.1j
    e2 = _modal_err(2, k, n, beta)
    e3 = _modal_err(3, k, n, beta)
    assert e3 < 0.05 and e3 < 0.6 * e2


def _solve_sphere(subdiv, k, beta=None):
    nodes, tris = synth.icosphere(subdiv)
    g = element_geometry(nodes, tris)
    A = op.dense(g, k, beta=beta, p=preset("paper"))
    b = op.rhs_plane_wave(g, k, [0, 0, 1])
    return op.lu_solve(A, b), g


def test_rigid_sphere_solution_converges():
    k = 1.0
    errs = []
    for s in (2, 3):
        p, g = _solve_sphere(s, k)
        ref = sphere.pressure(g["x"] / np.linalg.norm(g["x"], axis=1, keepdims=True), k)
        errs.append(np.linalg.norm(p - ref) / np.linalg.norm(ref))
    assert errs[1] < 5e-3
    assert errs[1] < 0.5 * errs[0]


def test_impedance_sphere_solution():
    k, beta = 2.0, 1.0
    errs = []
    for s, n in ((2, 320), (3, 1280)):
        p, g = _solve_sphere(s, k, beta=np.full(n, beta))
        ref = sphere.pressure(g["x"] / np.linalg.norm(g["x"], axis=1, keepdims=True), k, beta=beta)
        errs.append(np.linalg.norm(p - ref) / np.linalg.norm(ref))
    assert errs[1] < 3e-2 and errs[1] < 0.6 * errs[0]
    # a sign error in c_j (reflecting instead of absorbing) is far off
    ref_wrong = sphere.pressure(g["x"] / np.linalg.norm(g["x"], axis=1, keepdims=True), k, beta=-beta)
    assert np.linalg.norm(p - ref_wrong) / np.linalg.norm(ref_wrong) > 0.1


def test_field_points_match_series():
    k = 1.0
    p, g = _solve_sphere(3, k)
    pts = synth.points_on_sphere(12, 2.0, seed=5)
    M = field.field_matrix(g, pts, k, p=preset("paper"))
    pf = field.plane_wave(pts, k, [0, 0, 1]) + M @ p
    ref = sphere.pressure(pts, k)
    assert np.linalg.norm(pf - ref) / np.linalg.norm(ref) < 5e-3


def test_reciprocity_of_point_sources():
    k = 1.5
    nodes, tris = synth.icosphere(3)
    g = element_geometry(nodes, tris)
    A = op.dense(g, k, p=preset("paper"))
    xa = np.array([0.0, 0.0, 1.6])
    xb = np.array([1.3, 0.4, -0.9])
    pa = op.lu_solve(A, op.rhs_point_source(g, k, xa))
    pb = op.lu_solve(A, op.rhs_point_source(g, k, xb))
    Mb = field.field_matrix(g, xb[None], k, p=preset("paper"))
    Ma = field.field_matrix(g, xa[None], k, p=preset("paper"))
    p_ab = field.point_source(xb[None], k, xa) + Mb @ pa
    p_ba = field.point_source(xa[None], k, xb) + Ma @ pb
    assert abs(p_ab[0] - p_ba[0]) < 5e-3 * abs(p_ab[0])


@pytest.mark.parametrize("n,beta", [(0, 0.0), (1, 0.0), (0, 0.8 + 0.1j)])
def test_modal_eigenvalues_converge_other_coupling_sign(n, beta):
    # gamma = -i/k: the same closed form with the coupling's sign flipped
    # (errors are already near the constant-element stall on the coarse
    # mesh, so the check is a small and decreasing error)
    k = 2.0
    e2 = _modal_err(2, k, n, beta, gamma=-1j / k)
    e3 = _modal_err(3, k, n, beta, gamma=-1j / k)
    assert e3 < 0.02 and e3 < 0.8 * e2


def test_coupling_from_preset():
    k = 3.0
    assert op.coupling(k, None, preset("paper")) == 1j / k
    assert op.coupling(k, None, preset("tight")) == -1j / k
    assert op.coupling(k, 0.5j, preset("tight")) == 0.5j
    assert op.coupling(k) == 1j / k


def test_coupling_sign_and_spectrum():
    """On the sphere both signs give the same |lambda_n|; with gamma = -i/k
    every modal eigenvalue has a positive real part, while gamma = +i/k
    sends the propagating degrees (n < ka) around the origin.  The discrete
    operator of a non-spherical body shows the same split."""
    k = 27.7
    lp = np.array([sphere.bm_eigenvalue(n, k, gamma=1j / k) for n in range(70)])
    lm = np.array([sphere.bm_eigenvalue(n, k, gamma=-1j / k) for n in range(70)])
    assert np.allclose(np.abs(lp), np.abs(lm), rtol=1e-12)
    assert lm.real.min() > 0.4
    assert lp.real.min() < -0.5
    nodes, tris, _, _ = synth.graded_ellipsoid_bump(freq=6, grading=1.0, bump_height=0.0)
    g = element_geometry(nodes, tris)
    kk = 2 * np.pi * 4000.0 / 343.0
    ev_m = np.linalg.eigvals(op.dense(g, kk, p=preset("paper"), gamma=-1j / kk))
    ev_p = np.linalg.eigvals(op.dense(g, kk, p=preset("paper"), gamma=1j / kk))
    assert ev_m.real.min() > 0.3
    assert ev_p.real.min() < 0.0
