"""Pins for oracle.kernels: H, H', E against finite differences of G."""

import numpy as np
import pytest

from oracle.kernels import kernels, green


@pytest.mark.parametrize("k", [0.0, 1.0, 7.5])
def test_derivatives_match_finite_differences(k):
    rng = np.random.default_rng(11)
    for _ in range(20):
        x = rng.standard_normal(3)
        y = x + rng.standard_normal(3) * 0.7 + 0.3
        nx = rng.standard_normal(3)
        nx /= np.linalg.norm(nx)
        ny = rng.standard_normal(3)
        ny /= np.linalg.norm(ny)
        G, H, Hp, E = kernels(x, nx, y, ny, k)
        h = 1e-4
        Gf = lambda xx, yy: green(xx, yy, k)
        H_fd = (Gf(x, y + h * ny) - Gf(x, y - h * ny)) / (2 * h)
        Hp_fd = (Gf(x + h * nx, y) - Gf(x - h * nx, y)) / (2 * h)
        E_fd = (Gf(x + h * nx, y + h * ny) - Gf(x + h * nx, y - h * ny)
                - Gf(x - h * nx, y + h * ny) + Gf(x - h * nx, y - h * ny)) / (4 * h * h)
        assert G == pytest.approx(Gf(x, y), rel=1e-14)
        scale = abs(G) + abs(H) + abs(Hp) + abs(E)
        assert abs(H - H_fd) < 1e-7 * scale
        assert abs(Hp - Hp_fd) < 1e-7 * scale
        assert abs(E - E_fd) < 1e-6 * scale


def test_symmetry_relations():
    # H'(x, y) with n_x equals H(y, x) with the same normal at y: swapping the
    # roles of x and y flips the sign of R.
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(3), rng.standard_normal(3) + 2.0
    n = rng.standard_normal(3)
    n /= np.linalg.norm(n)
    _, _, Hp, _ = kernels(x, n, y, n, 2.0)
    _, H, _, _ = kernels(y, n, x, n, 2.0)
    assert Hp == pytest.approx(H, rel=1e-13)
