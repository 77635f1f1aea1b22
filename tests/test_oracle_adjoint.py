"""Pins for the oracle's admittance gradient (oracle/adjoint.py).

* A(c) = A0 + V diag(c): two dense assemblies of the whole operator (with and
  without admittance) against the directly assembled V.
* dJ/dY against central finite differences, with the operator, the right-hand
  side and the field map re-assembled from scratch at each perturbed Y; a
  dropped term of the adjoint formula, a wrong conjugation or sign fails here.
"""

import numpy as np

from oracle import adjoint, presets
from oracle.geometry import element_geometry
from oracle.operator import dense
from synth.meshes import icosphere
from synth.vectors import points_on_sphere, uniform01

RHO_C = 1.21 * 343.0


def _setup(k=2.0, npts=8, seed=3):
    nodes, tris = icosphere(1)
    N = tris.shape[0]
    Y = (1.0 + 0.5 * uniform01(N, seed)) / RHO_C
    pts = points_on_sphere(npts, 2.0, seed + 1)
    return nodes, tris, Y, pts, k


def test_operator_is_affine_in_c():
    nodes, tris, Y, _, k = _setup()
    geom = element_geometry(nodes, tris)
    p = presets.preset("paper")
    beta = RHO_C * Y.astype(np.complex128) * (1.0 + 0.3j)
    A1 = dense(geom, k, beta=beta, p=p)
    A0 = dense(geom, k, beta=None, p=p)
    V = adjoint.dense_dc(geom, k, p)
    c = -1j * k * beta
    err = np.abs(A1 - A0 - V * c[None, :]).max()
    assert err < 1e-12 * np.abs(A1).max()


def test_gradient_matches_central_differences():
    nodes, tris, Y, pts, k = _setup()
    p = presets.preset("paper")
    source = ("plane", (0.3, -0.2, 1.0), 1.0 + 0.5j)
    J, g, _ = adjoint.gradient(nodes, tris, Y, k, RHO_C, pts, source, p)
    assert J > 0.0

    def J_at(Yp):
        return adjoint.objective(nodes, tris, Yp, k, RHO_C, pts, source, p)[0]

    h = 1e-5 / RHO_C
    rng = np.random.default_rng(7)
    for e in rng.choice(Y.size, 4, replace=False):
        Yp, Ym = Y.copy(), Y.copy()
        Yp[e] += h
        Ym[e] -= h
        fd = (J_at(Yp) - J_at(Ym)) / (2 * h)
        assert abs(fd - g[e]) <= 1e-6 * np.abs(g).max(), (e, fd, g[e])
    d = rng.standard_normal(Y.size)
    fd = (J_at(Y + h * d) - J_at(Y - h * d)) / (2 * h)
    assert abs(fd - g @ d) <= 1e-6 * abs(g) @ np.abs(d)


def test_point_source_gradient_matches_central_differences():
    nodes, tris, Y, pts, k = _setup(k=1.3, npts=5, seed=11)
    p = presets.preset("paper")
    source = ("point", (0.0, 0.0, 1.4), 2.0)
    J, g, _ = adjoint.gradient(nodes, tris, Y, k, RHO_C, pts, source, p)
    h = 1e-5 / RHO_C
    d = np.random.default_rng(9).standard_normal(Y.size)
    Jp = adjoint.objective(nodes, tris, Y + h * d, k, RHO_C, pts, source, p)[0]
    Jm = adjoint.objective(nodes, tris, Y - h * d, k, RHO_C, pts, source, p)[0]
    fd = (Jp - Jm) / (2 * h)
    assert abs(fd - g @ d) <= 1e-6 * abs(g) @ np.abs(d)
