"""Pins of the plane-quadrilateral oracle (oracle/quad.py).

* Product rule (Sec. 3.1.4, m x m Gauss on the reference square): exact
  monomial integrals over a rectangle up to degree 2m - 1 per variable (and
  not 2m); on a plane trapezoid (non-affine bilinear map) the area and the
  first moments equal the polygon formulas.
* Self terms (Sec. 3.1.1-3.1.2, eight Duffy sub-triangles and four edges):
  with the collocation node x inside the plane polygon and rho(t) the
  distance from x to the boundary in direction t,
      G_ii = 1/(4 pi i k) int_0^{2 pi} (exp(i k rho) - 1) dt,
      E_ii = 1/(4 pi)     int_0^{2 pi} (i k - exp(i k rho)/rho) dt
  (k = 0: 1/(4 pi) int rho dt and -1/(4 pi) int 1/rho dt), by scipy quad.
* Off-diagonal integrals of a quadrilateral equal the sum over its two
  triangles computed by the triangle rules (a different rule family on the
  same region), at converged tolerance, from far, nearly singular and
  in-plane points.
* A rigid sphere of plane trapezoids with triangles at the poles (a mixed
  mesh) solves the plane-wave problem to within the first-order
  discretisation error of the analytic series, and the error falls with the
  mesh size.
"""

import math

import numpy as np
import pytest
from scipy.integrate import quad

import synth
from oracle import operator as op
from oracle import sphere
from oracle import quad as oq
from oracle.integrals import offdiag_integrals
from oracle.presets import preset


def _embed(P2d, origin, e1, e2):
    return np.array([origin + a * e1 + b * e2 for a, b in P2d])


def _frame():
    e1 = np.array([0.8, 0.1, -0.3])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(np.array([0.2, 0.7, 0.4]), e1)
    e2 /= np.linalg.norm(e2)
    return np.array([0.3, -0.2, 0.5]), e1, e2


def test_product_rule_rectangle_exactness():
    x0, x1, y0, y1 = -0.3, 0.9, 0.2, 1.1
    V = np.array([[x0, y0, 0.0], [x1, y0, 0.0], [x1, y1, 0.0], [x0, y1, 0.0]])
    for m in (1, 2, 3, 5):
        xi, eta, w = oq.product_rule(m)
        y, J = oq.bilinear(V, xi, eta)
        for a in range(0, 2 * m + 1):
            for b in (0, 2 * m - 1):
                exact = (x1 ** (a + 1) - x0 ** (a + 1)) / (a + 1) * (y1 ** (b + 1) - y0 ** (b + 1)) / (b + 1)
                got = np.sum(w * J * y[:, 0] ** a * y[:, 1] ** b)
                if a <= 2 * m - 1:
                    assert got == pytest.approx(exact, rel=1e-13, abs=1e-15)
                elif b == 0:
                    assert abs(got - exact) > 1e-8 * abs(exact)


def test_product_rule_trapezoid_moments():
    o, e1, e2 = _frame()
    P2 = np.array([[0.0, 0.0], [1.3, 0.1], [1.0, 0.9], [0.15, 0.7]])
    V = _embed(P2, o, e1, e2)
    # shoelace area and centroid of the polygon
    xs, ys = P2[:, 0], P2[:, 1]
    cr = xs * np.roll(ys, -1) - np.roll(xs, -1) * ys
    area = 0.5 * cr.sum()
    cx = np.sum((xs + np.roll(xs, -1)) * cr) / (6 * area)
    cy = np.sum((ys + np.roll(ys, -1)) * cr) / (6 * area)
    xi, eta, w = oq.product_rule(2)
    y, J = oq.bilinear(V, xi, eta)
    assert np.sum(w * J) == pytest.approx(area, rel=1e-14)
    assert oq.quad_area(V) == pytest.approx(area, rel=1e-14)
    c3 = np.sum((w * J)[:, None] * y, axis=0) / area
    assert np.allclose(c3, o + cx * e1 + cy * e2, rtol=0, atol=1e-14)


def _polar_self_polygon(P2d, x2d, k):
    """Closed forms above for x2d inside the convex polygon P2d (n, 2)."""
    v = P2d - x2d
    edges = [(v[a], v[(a + 1) % len(v)]) for a in range(len(v))]

    def rho(t):
        u = np.array([np.cos(t), np.sin(t)])
        best = np.inf
        for a, b in edges:
            d = b - a
            det = u[0] * (-d[1]) - u[1] * (-d[0])
            if abs(det) < 1e-300:
                continue
            r = (a[0] * (-d[1]) - a[1] * (-d[0])) / det
            s = (u[0] * a[1] - u[1] * a[0]) / det
            if r > 0 and -1e-12 <= s <= 1 + 1e-12:
                best = min(best, r)
        return best

    ang = np.sort(np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * np.pi))
    pts = np.concatenate([[0.0], ang, [2 * np.pi]])

    def integ(f):
        return sum(quad(f, a, b, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
                   for a, b in zip(pts[:-1], pts[1:]) if b - a > 1e-15)

    if k == 0.0:
        return integ(rho) / (4 * np.pi), -integ(lambda t: 1.0 / rho(t)) / (4 * np.pi)
    G = (integ(lambda t: np.cos(k * rho(t)) - 1.0) + 1j * integ(lambda t: np.sin(k * rho(t)))) / (4j * np.pi * k)
    E = (integ(lambda t: -np.cos(k * rho(t)) / rho(t))
         + 1j * integ(lambda t: k - np.sin(k * rho(t)) / rho(t))) / (4 * np.pi)
    return G, E


@pytest.mark.parametrize("k", [0.0, 1.0, 12.0, 40.0])
def test_self_quad_matches_polar_integrals(k):
    o, e1, e2 = _frame()
    P2 = np.array([[0.0, 0.0], [1.3, 0.1], [1.0, 0.9], [0.15, 0.7]]) * 0.2
    V = _embed(P2, o, e1, e2)[None]
    g = oq.mixed_geometry(V[0], np.array([[0, 1, 2, 3]]))
    x2 = P2.mean(axis=0)
    assert np.allclose(g["x"][0], o + x2[0] * e1 + x2[1] * e2, atol=1e-15)
    Gp, Ep = _polar_self_polygon(P2, x2, k)
    Gs, Es = oq.self_quad(g["V"], g["x"], g["n"], k, preset("tight"))
    assert abs(Gs[0] - Gp) < 1e-10 * abs(Gp)
    assert abs(Es[0] - Ep) < 1e-9 * abs(Ep)
    # the paper's 4 x 4 Duffy and 4 x 3 edge rules: a few digits
    Gs4, Es4 = oq.self_quad(g["V"], g["x"], g["n"], k, preset("paper"))
    assert abs(Gs4[0] - Gp) < 1e-3 * abs(Gp)
    assert abs(Es4[0] - Ep) < 2e-2 * abs(Ep)


@pytest.mark.parametrize("k", [0.5, 9.0])
def test_quad_integrals_equal_two_triangles(k):
    o, e1, e2 = _frame()
    P2 = np.array([[0.0, 0.0], [1.3, 0.1], [1.0, 0.9], [0.15, 0.7]]) * 0.3
    V = _embed(P2, o, e1, e2)
    g = oq.mixed_geometry(V, np.array([[0, 1, 2, 3]]))
    ny = g["n"][0]
    c = g["x"][0]
    pts = np.array([c + 2.0 * ny, c + 0.05 * ny + 0.02 * e1, c + 0.4 * e1 + 0.5 * e2 + 0.01 * ny,
                    o + 0.6 * e1 - 0.05 * e2, c + 3.0 * e1 - 1.0 * ny])
    nx = np.tile(np.array([0.3, -0.4, 0.866]), (len(pts), 1))
    p = preset("tight", quad_eps=1e-13)
    Q = oq.offdiag_quad(pts, nx, np.repeat(V[None], len(pts), 0), np.tile(ny, (len(pts), 1)), k, p)
    tri = np.zeros_like(Q)
    for a, b, cc in ((0, 1, 2), (0, 2, 3)):
        A = 0.5 * np.linalg.norm(np.cross(V[b] - V[a], V[cc] - V[a]))
        rep = lambda v: np.tile(v, (len(pts), 1))
        tri += offdiag_integrals(pts, nx, rep(V[a]), rep(V[b]), rep(V[cc]), rep(ny), np.full(len(pts), A), k, p)
    # per integral, relative to its largest value over the points (the in-plane
    # point has I^H = 0 exactly)
    assert np.max(np.abs(Q - tri) / np.max(np.abs(tri), axis=1, keepdims=True)) < 1e-9


def _sphere_error(n_theta, n_phi, k):
    nodes, el = synth.uv_sphere(n_theta, n_phi)
    g = oq.mixed_geometry(nodes, el)
    p = preset("tight")
    A = oq.dense(g, k, p=p)
    b = op.rhs_plane_wave(g, k, [0.0, 0.0, 1.0], p=p)
    ph = op.lu_solve(A, b)
    an = sphere.pressure(g["x"] / np.linalg.norm(g["x"], axis=1, keepdims=True), k)
    return np.linalg.norm(ph - an) / np.linalg.norm(an), g


def test_mixed_sphere_rigid_series():
    k = 2.0
    e1, g1 = _sphere_error(8, 16, k)
    e2, g2 = _sphere_error(16, 32, k)
    assert g1["is_quad"].sum() == 16 * 6 and (~g1["is_quad"]).sum() == 32
    assert e2 < 0.015 and e2 < 0.4 * e1, (e1, e2)  # 0.0385 -> 0.0106
