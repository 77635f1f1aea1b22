"""The stored c2 oracle results (tests/golden/c2_sphere20480.npz) against a
fresh computation by the oracle and against the analytic rigid-sphere series:
sampled rows of the dense operator reproduce the stored A x, the stored
right-hand side is the oracle's, and the stored LU pressure lies within the
first-order discretisation error of the series solution (Sec. 5.1.2 measures
the same order on its sphere meshes)."""

import math
import os

import numpy as np

import synth
from oracle import operator as op
from oracle import sphere
from oracle.geometry import element_geometry
from oracle.presets import preset

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c2_sphere20480.npz")


def test_golden_c2_matches_oracle():
    z = np.load(GOLDEN)
    nodes, tris = synth.icosphere(5)
    g = element_geometry(nodes, tris)
    N = len(tris)
    k = 2 * math.pi / (6.0 * synth.mean_edge_length(nodes, tris))
    assert int(z["N"]) == N and float(z["k"]) == k
    x = synth.complex_normal(N, seed=int(z["x_seed"]))
    rows = np.random.default_rng(11).choice(N, 6, replace=False)
    Ar = op.rows(g, rows, k, p=preset("tight", quad_eps=float(z["quad_eps"])))
    y = z["y_ax"]
    assert np.max(np.abs(Ar @ x - y[rows])) < 1e-12 * np.max(np.abs(y))
    b = op.rhs_plane_wave(g, k, [0.0, 0.0, 1.0], p=preset("tight"))
    assert np.array_equal(b, z["b"])
    # the LU solution solves the stored system row by row ...
    p = z["p_lu"]
    assert np.linalg.norm(Ar @ p - b[rows]) < 1e-10 * np.linalg.norm(b[rows])
    # ... and is the rigid sphere's pressure up to the discretisation error
    an = sphere.pressure(g["x"] / np.linalg.norm(g["x"], axis=1, keepdims=True), k)
    err = np.linalg.norm(p - an) / np.linalg.norm(an)
    assert 1e-3 < err < 3e-2
