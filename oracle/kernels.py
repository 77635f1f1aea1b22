"""Helmholtz kernels (oracle; test infrastructure only).

G(x, y) = exp(i k r) / (4 pi r), r = |x - y|  (Sec. 2.1, after Eq. (BIE_I)).
H  = dG/dn_y   (Sec. 2.1),
H' = dG/dn_x   and  E = d2G/(dn_x dn_y)  (Sec. 2.5, after Eq. (dBIE)).

Written out with R = y - x, Rh = R / r:
    dG/dr = G (i k - 1/r)
    H  =  G (i k - 1/r) (Rh . n_y)
    H' = -G (i k - 1/r) (Rh . n_x)
    E  = -G [ (3/r^2 - 3 i k / r - k^2) (Rh . n_x)(Rh . n_y)
              + (i k - 1/r) (n_x . n_y) / r ]

Pinned by: tests/test_oracle_kernels.py (central finite differences of G in
x along n_x and in y along n_y).
"""

import numpy as np

FOUR_PI = 4.0 * np.pi


def kernels(x, nx, y, ny, k):
    """Evaluate (G, H, H', E) for broadcastable arrays of points/normals.

    x, nx, y, ny: (..., 3) float64; k: real wavenumber.
    Returns four complex arrays of the broadcast shape (...)."""
    R = y - x
    r = np.sqrt(np.sum(R * R, axis=-1))
    inv_r = 1.0 / r
    G = np.exp(1j * k * r) * inv_r / FOUR_PI
    rn_y = np.sum(R * ny, axis=-1) * inv_r
    rn_x = np.sum(R * nx, axis=-1) * inv_r
    nn = np.sum(nx * ny, axis=-1)
    a = 1j * k - inv_r
    H = G * a * rn_y
    Hp = -G * a * rn_x
    E = -G * ((3.0 * inv_r * inv_r - 3j * k * inv_r - k * k) * rn_x * rn_y
              + a * nn * inv_r)
    return G, H, Hp, E


def green(x, y, k):
    """G(x, y) alone."""
    R = y - x
    r = np.sqrt(np.sum(R * R, axis=-1))
    return np.exp(1j * k * r) / (FOUR_PI * r)
