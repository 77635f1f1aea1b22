"""Pins for oracle.integrals against mathematics that does not use its rules.

* Self terms: with the collocation node x inside a flat triangle and rho(t)
  the distance from x to the boundary along the in-plane direction at angle
  t, the radial integrals are elementary:
      G_ii = 1/(4 pi i k) int_0^{2 pi} (exp(i k rho) - 1) dt   (k -> 0: 1/(4 pi) int rho dt)
      E_ii = 1/(4 pi)     int_0^{2 pi} (i k - exp(i k rho)/rho) dt
  (the E form is the Hadamard finite part: the inner radial integral of the
  in-plane hypersingular kernel is (1 - exp(ik rho))/rho + ik - 1/rho).
  The angular integrals are done by scipy's adaptive quad.
* Static equilateral values: int G0 = sqrt(3) h ln(2 + sqrt 3)/(4 pi),
  E0 = -9/(2 pi h).
* Regular and nearly singular pairs: scipy dblquad over the triangle.
"""

import numpy as np
import pytest
from scipy.integrate import quad, dblquad

import synth
from oracle.geometry import element_geometry
from oracle.integrals import offdiag_integrals, self_integrals, estimator_order, SubdivisionError
from oracle.kernels import kernels
from oracle.presets import preset


def _frame(P):
    e1 = P[1] - P[0]
    e1 /= np.linalg.norm(e1)
    n = np.cross(P[1] - P[0], P[2] - P[0])
    n /= np.linalg.norm(n)
    e2 = np.cross(n, e1)
    return e1, e2


def _polar_pieces(P, x):
    """Angular breakpoints and rho(t) for x inside triangle P (3,3)."""
    e1, e2 = _frame(P)
    v = np.array([[(p - x) @ e1, (p - x) @ e2] for p in P])

    def rho(t):
        u = np.array([np.cos(t), np.sin(t)])
        best = np.inf
        for a, b in ((v[0], v[1]), (v[1], v[2]), (v[2], v[0])):
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
    return rho, pts


def polar_self(P, x, k):
    rho, pts = _polar_pieces(P, x)

    def integ(f):
        tot = 0.0
        for a, b in zip(pts[:-1], pts[1:]):
            if b - a < 1e-15:
                continue
            tot += quad(f, a, b, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
        return tot

    if k == 0.0:
        G = integ(rho) / (4 * np.pi)
        E = -integ(lambda t: 1.0 / rho(t)) / (4 * np.pi)
        return G, E
    gre = integ(lambda t: np.cos(k * rho(t)) - 1.0)
    gim = integ(lambda t: np.sin(k * rho(t)))
    G = (gre + 1j * gim) / (4j * np.pi * k)
    ere = integ(lambda t: -np.cos(k * rho(t)) / rho(t))
    eim = integ(lambda t: k - np.sin(k * rho(t)) / rho(t))
    E = (ere + 1j * eim) / (4 * np.pi)
    return G, E


def _geom_of(P):
    P = np.asarray(P, dtype=np.float64)
    return element_geometry(P, np.array([[0, 1, 2]]))


def test_static_equilateral_closed_form():
    h = 0.37
    P = np.array([[0, 0, 0], [h, 0, 0], [h / 2, h * np.sqrt(3) / 2, 0]])
    g = _geom_of(P)
    Gs, Es = self_integrals(g, 0.0, preset("tight"))
    assert Gs[0].real == pytest.approx(np.sqrt(3) * h * np.log(2 + np.sqrt(3)) / (4 * np.pi), rel=1e-12)
    assert Es[0].real == pytest.approx(-9 / (2 * np.pi * h), rel=1e-10)
    Gp, Ep = polar_self(P, g["x"][0], 0.0)
    assert Gp == pytest.approx(Gs[0].real, rel=1e-11)
    assert Ep == pytest.approx(Es[0].real, rel=1e-11)


@pytest.mark.parametrize("k", [0.0, 1.0, 12.0, 40.0])
def test_self_terms_match_polar_integrals(k):
    # a scalene, tilted triangle
    P = np.array([[0.1, -0.2, 0.3], [0.9, 0.1, 0.25], [0.35, 0.6, -0.1]]) * 0.2
    g = _geom_of(P)
    Gp, Ep = polar_self(P, g["x"][0], k)
    Gs, Es = self_integrals(g, k, preset("tight"))
    assert abs(Gs[0] - Gp) < 1e-10 * abs(Gp)
    assert abs(Es[0] - Ep) < 1e-9 * abs(Ep)
    # the paper's 4x4 / 4x3 rules are accurate to a few digits on this shape
    Gs4, Es4 = self_integrals(g, k, preset("paper"))
    assert abs(Gs4[0] - Gp) < 1e-3 * abs(Gp)
    assert abs(Es4[0] - Ep) < 2e-2 * abs(Ep)


def _brute(x, nx, P, ny, k, which):
    P0, P1, P2 = P
    A2 = np.linalg.norm(np.cross(P1 - P0, P2 - P0))

    def f(t, s, part):
        y = P0 + s * (P1 - P0) + t * (P2 - P0)
        v = kernels(x, nx, y, ny, k)[which] * A2
        return v.real if part == 0 else v.imag

    re = dblquad(lambda t, s: f(t, s, 0), 0, 1, 0, lambda s: 1 - s, epsabs=1e-14, epsrel=1e-12)[0]
    im = dblquad(lambda t, s: f(t, s, 1), 0, 1, 0, lambda s: 1 - s, epsabs=1e-14, epsrel=1e-12)[0]
    return re + 1j * im


def test_offdiagonal_against_adaptive_quadrature():
    nodes, tris = synth.icosphere(2)
    g = element_geometry(nodes, tris)
    i = 0
    d = np.linalg.norm(g["x"] - g["x"][i], axis=1) / np.sqrt(g["A"])
    order = np.argsort(d)
    picks = [order[1], order[3], order[12], order[60], order[-1]]  # adjacent ... far
    k = 6.0
    for j in picks:
        P = (g["P0"][j], g["P1"][j], g["P2"][j])
        I = offdiag_integrals(g["x"][[i]], g["n"][[i]], g["P0"][[j]], g["P1"][[j]],
                              g["P2"][[j]], g["n"][[j]], g["A"][[j]], k, preset("tight"))
        Ip = offdiag_integrals(g["x"][[i]], g["n"][[i]], g["P0"][[j]], g["P1"][[j]],
                               g["P2"][[j]], g["n"][[j]], g["A"][[j]], k, preset("paper"))
        for w in range(4):
            ref = _brute(g["x"][i], g["n"][i], P, g["n"][j], k, w)
            scale = abs(ref) + 1e-3 * abs(_brute(g["x"][i], g["n"][i], P, g["n"][j], k, 0))
            assert abs(I[w, 0] - ref) < 2e-7 * scale, (j, w, I[w, 0], ref)
            assert abs(Ip[w, 0] - ref) < 3e-2 * scale, (j, w, Ip[w, 0], ref)


def test_self_H_terms_are_exactly_zero_in_plane():
    # for any in-plane y, (y - x) . n = 0 so H and H' vanish identically
    nodes, tris = synth.icosphere(1)
    g = element_geometry(nodes, tris)
    for e in range(5):
        y = g["P0"][e] * 0.3 + g["P1"][e] * 0.5 + g["P2"][e] * 0.2
        G, H, Hp, _ = kernels(g["x"][e], g["n"][e], y, g["n"][e], 3.0)
        r = np.linalg.norm(y - g["x"][e])
        scale = abs(G) * abs(3j - 1.0 / r)
        assert abs(H) < 1e-13 * scale and abs(Hp) < 1e-13 * scale


def test_estimator_orders():
    # thresholds implied by the three estimates at the paper tolerance
    m = estimator_order(np.array([1.3, 2.0, 3.0, 5.0, 15.0, 17.0, 100.0]), 1e-3)
    assert list(m) == [8, 5, 3, 2, 2, 1, 1]


def test_subdivision_depth_error():
    # a collocation node sitting on the source element's plane, almost on its
    # vertex, never satisfies r~ >= 1.3 for small enough sub-elements
    P = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    g = _geom_of(P)
    x = np.array([[1e-9, 1e-9, 0.0]])
    with pytest.raises(SubdivisionError):
        offdiag_integrals(x, g["n"], g["P0"], g["P1"], g["P2"], g["n"], g["A"], 1.0,
                          preset("paper"))
