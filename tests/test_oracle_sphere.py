"""Pins for oracle.sphere: internal identities of the closed forms."""

import numpy as np
import pytest
from scipy.special import eval_legendre, spherical_jn

from oracle import sphere


@pytest.mark.parametrize("k", [0.5, 1.0, 3.696, 14.784])
def test_series_equals_wronskian_closed_form(k):
    ct = np.linspace(-1, 1, 41)
    pts = np.stack([np.sqrt(1 - ct ** 2), np.zeros_like(ct), ct], axis=1)
    a = sphere.pressure(pts, k)
    b = sphere.surface_pressure_rigid(ct, k)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("k", [1.0, 5.0])
def test_modal_solution_reproduces_series(k):
    # rigid: phi_n = i^n (2n+1) (j_n - gamma k j_n') / lambda_n
    gamma = 1j / k
    ct = np.linspace(-1, 1, 17)
    tot = np.zeros_like(ct, dtype=complex)
    for n in range(sphere.n_terms(k) + 1):
        rhs = (1j ** n) * (2 * n + 1) * (spherical_jn(n, k) - gamma * k * spherical_jn(n, k, True))
        tot += rhs / sphere.bm_eigenvalue(n, k) * eval_legendre(n, ct)
    assert np.max(np.abs(tot - sphere.surface_pressure_rigid(ct, k))) < 1e-12


@pytest.mark.parametrize("k", [1.0, 4.0])
def test_modal_impedance_solution_reproduces_series(k):
    beta = 0.7 + 0.2j
    gamma = 1j / k
    ct = np.linspace(-1, 1, 9)
    tot = np.zeros_like(ct, dtype=complex)
    for n in range(sphere.n_terms(k) + 1):
        rhs = (1j ** n) * (2 * n + 1) * (spherical_jn(n, k) - gamma * k * spherical_jn(n, k, True))
        tot += rhs / sphere.bm_eigenvalue(n, k, beta=beta) * eval_legendre(n, ct)
    pts = np.stack([np.sqrt(1 - ct ** 2), np.zeros_like(ct), ct], axis=1)
    ref = sphere.pressure(pts, k, beta=beta)
    assert np.max(np.abs(tot - ref)) < 1e-11 * np.max(np.abs(ref))


def test_coupling_sign_does_not_change_modulus():
    for k in (0.7, 3.0, 11.0):
        for n in range(6):
            a = sphere.bm_eigenvalue(n, k, gamma=1j / k)
            b = sphere.bm_eigenvalue(n, k, gamma=-1j / k)
            assert abs(abs(a) - abs(b)) < 1e-13 * abs(a)


def test_static_limits():
    k = 1e-4
    for n in range(5):
        S, K, W = sphere.modal(n, k)
        assert S.real == pytest.approx(1.0 / (2 * n + 1), rel=1e-6)
        assert K.real == pytest.approx(-1.0 / (2 * (2 * n + 1)), rel=1e-6, abs=1e-9)
        assert W.real == pytest.approx(-n * (n + 1) / (2 * n + 1), rel=1e-6, abs=1e-7)


def test_impedance_absorbs():
    # exterior admittance with Re beta > 0 takes energy out of the field:
    # Re(conj(p) v) <= 0 with v = -beta p / (rho c)
    k = 2.0
    beta = 1.0
    ct = np.linspace(-1, 1, 11)
    pts = np.stack([np.sqrt(1 - ct ** 2), np.zeros_like(ct), ct], axis=1)
    p = sphere.pressure(pts, k, beta=beta)
    v = -beta * p
    assert np.all(np.real(np.conj(p) * v) <= 0)
