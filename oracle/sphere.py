"""Closed-form sphere results (oracle; test infrastructure only).

The paper checks against the analytic solution for a plane wave on a
sound-hard sphere (Sec. 5.1); its textbook formula is not reproduced in the
paper, so the series is derived here from the plane-wave expansion
exp(i k r cos t) = sum_n i^n (2n+1) j_n(k r) P_n(cos t) with exp(-i w t)
time dependence and h_n = h_n^(1):

    p(r, t) = sum_n i^n (2n+1) [ j_n(k r) + A_n h_n(k r) ] P_n(cos t),
    A_n = -( j_n'(x) + i beta j_n(x) ) / ( h_n'(x) + i beta h_n(x) ),  x = k a,

from dp/dr = -i k beta p on r = a (exterior admittance, v = -Y p,
beta = rho c Y; beta = 0 is sound-hard).  On the sound-hard surface the
Wronskian j_n h_n' - j_n' h_n = i / x^2 gives
p(a, t) = sum_n i^n (2n+1) i / (x^2 h_n'(x)) P_n(cos t).

Modal eigenvalues on a sphere of radius a for spherical harmonics of
degree n (G = exp(ikr)/(4 pi r)):
    single layer  S_n = i k a^2 j_n h_n
    double layer  K_n = K'_n = 1/2 + i x^2 j_n h_n'   (principal value)
    hypersingular W_n = i k^3 a^2 j_n' h_n'
and the Burton-Miller operator of Eq. (SystemI) has eigenvalue
    lambda_n = (1 - gamma c)/2 - K_n + gamma W_n + (S_n - gamma K'_n) c.

Pinned by: tests/test_oracle_sphere.py (series against the Wronskian
closed form, modal solution against the series, static limits).
"""

import numpy as np
from scipy.special import spherical_jn, spherical_yn, eval_legendre


def _h(n, x, derivative=False):
    return spherical_jn(n, x, derivative) + 1j * spherical_yn(n, x, derivative)


def n_terms(x):
    return int(x + 10.0 * x ** (1.0 / 3.0) + 10)


def pressure(points, k, a=1.0, beta=0.0, d=(0.0, 0.0, 1.0), P0=1.0, nmax=None):
    """Total pressure of a plane wave P0 exp(i k d.x) scattered by a sphere
    of radius ``a`` centred at the origin with uniform admittance ``beta``,
    evaluated at ``points`` (M,3) with |x| >= a."""
    pts = np.asarray(points, dtype=np.float64)
    r = np.linalg.norm(pts, axis=1)
    ct = (pts @ np.asarray(d, dtype=np.float64)) / r
    x = k * a
    nmax = n_terms(max(x, k * r.max())) if nmax is None else nmax
    out = np.zeros(pts.shape[0], dtype=np.complex128)
    for n in range(nmax + 1):
        An = -(spherical_jn(n, x, True) + 1j * beta * spherical_jn(n, x)) / \
             (_h(n, x, True) + 1j * beta * _h(n, x))
        out += (1j ** n) * (2 * n + 1) * (spherical_jn(n, k * r) + An * _h(n, k * r)) \
            * eval_legendre(n, ct)
    return P0 * out


def surface_pressure_rigid(cos_t, k, a=1.0, P0=1.0, nmax=None):
    """Wronskian closed form of the sound-hard surface pressure."""
    x = k * a
    nmax = n_terms(x) if nmax is None else nmax
    out = np.zeros(np.shape(cos_t), dtype=np.complex128)
    for n in range(nmax + 1):
        out += (1j ** n) * (2 * n + 1) * 1j / (x * x * _h(n, x, True)) * eval_legendre(n, cos_t)
    return P0 * out


def modal(n, k, a=1.0):
    """(S_n, K_n, W_n) of the continuous operators on the sphere."""
    x = k * a
    jn, jd = spherical_jn(n, x), spherical_jn(n, x, True)
    hn, hd = _h(n, x), _h(n, x, True)
    S = 1j * k * a * a * jn * hn
    K = 0.5 + 1j * x * x * jn * hd
    W = 1j * k ** 3 * a * a * jd * hd
    return S, K, W


def bm_eigenvalue(n, k, a=1.0, beta=0.0, gamma=None):
    """Eigenvalue of the Burton-Miller operator of Eq. (SystemI) for degree n."""
    gamma = 1j / k if gamma is None else gamma
    c = -1j * k * beta
    S, K, W = modal(n, k, a)
    return 0.5 * (1.0 - gamma * c) - K + gamma * W + (S - gamma * K) * c
