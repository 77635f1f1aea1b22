"""Pins for oracle.rules: polynomial exactness of the triangle and edge rules."""

from math import factorial

import numpy as np
import pytest

from oracle.rules import conical, gauss_jacobi01, gauss_legendre01, edge_rule


def exact_monomial(a, b):
    # int over the reference triangle (0,0),(1,0),(0,1) of s^a t^b
    return factorial(a) * factorial(b) / factorial(a + b + 2)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 8])
def test_conical_rule_exact_to_degree_2m_minus_1(m):
    a, b, w = conical(m)
    # reference triangle P0 = 0, P1 = e1, P2 = e2: y = (a, b), area 1/2
    for deg in range(0, 2 * m):
        for p in range(deg + 1):
            q = deg - p
            val = np.sum(2 * 0.5 * w * a ** p * b ** q)
            assert val == pytest.approx(exact_monomial(p, q), rel=1e-12, abs=1e-15)
    # and not exact at degree 2m for some monomial (the order is sharp)
    errs = [abs(np.sum(w * a ** p * b ** (2 * m - p)) - exact_monomial(p, 2 * m - p))
            for p in range(2 * m + 1)]
    assert max(errs) > 1e-12


def test_conical_m1_is_centroid():
    a, b, w = conical(1)
    assert a[0] == pytest.approx(1 / 3)
    assert b[0] == pytest.approx(1 / 3)
    assert w[0] == pytest.approx(0.5)


def test_one_dimensional_rules():
    for n in range(1, 9):
        x, w = gauss_legendre01(n)
        for d in range(2 * n):
            assert np.sum(w * x ** d) == pytest.approx(1.0 / (d + 1), rel=1e-13)
        x, w = gauss_jacobi01(n)
        for d in range(2 * n):
            assert np.sum(w * x ** d) == pytest.approx(1.0 / (d + 2), rel=1e-13)
    t, w = edge_rule(4, 3)
    assert t.size == 12 and np.sum(w) == pytest.approx(1.0)
    # piecewise rule integrates a kinked function exactly when the kinks sit
    # on part boundaries
    f = lambda s: np.abs(s - 0.5) ** 3
    assert np.sum(w * f(t)) == pytest.approx(2 * (0.5 ** 4) / 4, rel=1e-13)
