"""The stored c4 oracle results (tests/golden/c4_sphere40500.npz: LU solutions
of the 40500-triangle sphere at three of the sweep's frequencies) against a
fresh computation by the oracle and against the analytic rigid-sphere series:
the stored right-hand sides are the oracle's, sampled rows of the operator
(recomputed with converged quadrature) are solved by the stored pressure, and
the pressure lies within the discretisation error of the series solution."""

import math
import os

import numpy as np
import pytest

import synth
from oracle import operator as op
from oracle import sphere
from oracle.geometry import element_geometry
from oracle.presets import preset

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c4_sphere40500.npz")


@pytest.fixture(scope="module")
def c4():
    if not os.path.exists(GOLDEN):
        pytest.skip("c4 golden file not generated (tests/golden/make_c4_golden.py)")
    z = np.load(GOLDEN)
    nodes, tris = synth.geodesic_sphere(45)
    g = element_geometry(nodes, tris)
    assert int(z["N"]) == len(tris)
    return z, g


def test_golden_c4_frequencies(c4):
    z, _ = c4
    for i in z["indices"]:
        f = 100.0 * 200.0 ** (int(i) / 63.0)
        assert float(z[f"k_{i}"]) == 2.0 * math.pi * f / float(z["c"])


@pytest.mark.parametrize("pos", [0, 1, 2])
def test_golden_c4_matches_oracle(c4, pos):
    z, g = c4
    i = int(z["indices"][pos])
    k = float(z[f"k_{i}"])
    b = op.rhs_plane_wave(g, k, [0.0, 0.0, 1.0], p=preset("mixed"))
    assert np.array_equal(b, z[f"b_{i}"])
    p = z[f"p_lu_{i}"]
    rows = np.random.default_rng(40 + i).choice(len(b), 2, replace=False)
    Ar = op.rows(g, rows, k, p=preset("mixed", quad_eps=float(z["quad_eps"])))
    assert np.linalg.norm(Ar @ p - b[rows]) < 1e-9 * np.linalg.norm(b[rows])
    an = sphere.pressure(g["x"] / np.linalg.norm(g["x"], axis=1, keepdims=True), k)
    err = np.linalg.norm(p - an) / np.linalg.norm(an)
    assert 1e-5 < err < 2e-2, err
