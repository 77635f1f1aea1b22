"""Quadrature rules (oracle; test infrastructure only).

Sec. 3.1 names the rules but prints no node tables, so these are the
readings used by both sides (each side computes its own nodes):

* ``gauss_legendre01(n)``  n-point Gauss-Legendre on [0, 1].
* ``gauss_jacobi01(n)``    n-point Gauss rule for weight xi on [0, 1]
                           (Jacobi alpha = 0, beta = 1 mapped from [-1, 1]).
* ``conical(m)``           regular triangle rule "based on m" (Sec. 3.1.4):
                           Stroud conical product of m-point Gauss-Jacobi in
                           xi and m-point Gauss-Legendre in eta, collapsed at
                           the first vertex:
                             y = P0 + xi (1 - eta) (P1 - P0) + xi eta (P2 - P0),
                             dA = 2 A xi dxi deta;
                           exact for polynomials of total degree <= 2m - 1;
                           m = 1 is the centroid rule.
* ``duffy_subtriangles``   singular rule of Sec. 3.1.1: the element is cut
                           into six triangles sharing the collocation node
                           (centroid joined to the three vertices and the
                           three edge midpoints); on each, the Duffy map
                           y = x + u [(Q1 - x) + v (Q2 - Q1)], dA = 2 A_s u du dv
                           with n x n Gauss-Legendre in u and v.
* ``edge_rule``            hypersingular edge integrals of Sec. 3.1.2: every
                           edge split into ``parts`` equal pieces with a
                           ``ng``-point Gauss-Legendre rule on each.

Pinned by: tests/test_oracle_rules.py (polynomial exactness against exact
monomial integrals over a triangle, weights sum to the area, the m = 1
node is the centroid).
"""

import numpy as np
from scipy.special import roots_jacobi


def gauss_legendre01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_jacobi01(n):
    # int_{-1}^{1} (1 + x) g(x) dx with xi = (1 + x)/2 equals 4 int_0^1 xi g dxi
    x, w = roots_jacobi(n, 0.0, 1.0)
    return 0.5 * (x + 1.0), 0.25 * w


def conical(m):
    """Return (a, b, w) of length m*m: the point is
    y = P0 + a (P1 - P0) + b (P2 - P0) and its weight is 2 A w."""
    xi, wx = gauss_jacobi01(m)
    eta, we = gauss_legendre01(m)
    XI, ETA = np.meshgrid(xi, eta, indexing="ij")
    W = np.outer(wx, we)
    a = XI * (1.0 - ETA)
    b = XI * ETA
    return a.ravel(), b.ravel(), W.ravel()


def duffy_subtriangles(P0, P1, P2, x):
    """The six sub-triangles (x, Q1, Q2) of the singular rule, as a list of
    (Q1, Q2) pairs in counter-clockwise order around the element."""
    M01 = 0.5 * (P0 + P1)
    M12 = 0.5 * (P1 + P2)
    M20 = 0.5 * (P2 + P0)
    return [(P0, M01), (M01, P1), (P1, M12), (M12, P2), (P2, M20), (M20, P0)]


def edge_rule(parts, ng):
    """Return (t, w) on [0, 1] for one edge: ``parts`` equal pieces with an
    ``ng``-point Gauss-Legendre rule on each (weights sum to 1)."""
    g, gw = gauss_legendre01(ng)
    t = (np.arange(parts)[:, None] + g[None, :]) / parts
    w = np.tile(gw, parts) / parts
    return t.ravel(), w
