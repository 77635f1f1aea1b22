"""Seeded random inputs (vectors, admittances, field points)."""

import numpy as np


def complex_normal(n, seed):
    """Complex vector whose real and imaginary parts are independent
    standard normals, from ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(n)
    im = rng.standard_normal(n)
    return re + 1j * im


def uniform01(n, seed):
    """Uniform(0, 1) samples from ``numpy.random.default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, n)


def points_on_sphere(n, radius, seed):
    """``n`` points uniformly distributed on the sphere of ``radius`` about
    the origin (normalised standard-normal directions)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d * radius
