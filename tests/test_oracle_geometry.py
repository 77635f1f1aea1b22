"""Pins of the oracle's flat-triangle geometry (Sec. 2.2-2.3, appendix "The
Mesh"): areas, unit outward normals and collocation points against values
fixed by hand computation and by the geometry of the sphere, not by the
oracle's own formulas."""

import math

import numpy as np
import pytest

import synth
from oracle.geometry import element_geometry


def test_hand_computed_triangles():
    # in-plane scalene triangle, counter-clockwise seen from +z:
    # base 3 along x, apex (1, 2): area 3, centroid (4/3, 2/3, 0), normal +z
    nodes = np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0], [1.0, 2.0, 0.0]])
    g = element_geometry(nodes, np.array([[0, 1, 2]]))
    assert g["A"][0] == pytest.approx(3.0, abs=1e-15)
    assert np.allclose(g["x"][0], [4.0 / 3.0, 2.0 / 3.0, 0.0], atol=1e-15)
    assert np.allclose(g["n"][0], [0.0, 0.0, 1.0], atol=1e-15)
    # a tilted one: edges (2, 0, 0) and (0, 3, 4) from (1, 2, 3); their cross
    # product is (0, -8, 6), length 10: area 5, normal (0, -4/5, 3/5)
    nodes = np.array([[1.0, 2.0, 3.0], [3.0, 2.0, 3.0], [1.0, 5.0, 7.0]])
    g = element_geometry(nodes, np.array([[0, 1, 2]]))
    assert g["A"][0] == pytest.approx(5.0, abs=1e-14)
    assert np.allclose(g["x"][0], [5.0 / 3.0, 3.0, 13.0 / 3.0], atol=1e-14)
    assert np.allclose(g["n"][0], [0.0, -0.8, 0.6], atol=1e-15)
    # clockwise order flips the normal, keeps area and centroid
    g2 = element_geometry(nodes, np.array([[0, 2, 1]]))
    assert np.allclose(g2["n"][0], -g["n"][0], atol=1e-15)
    assert g2["A"][0] == pytest.approx(5.0, abs=1e-14)
    assert np.allclose(g2["x"][0], g["x"][0], atol=1e-15)


def test_unit_regular_triangle():
    # equilateral triangle of side h: area sqrt(3) h^2 / 4
    h = 0.37
    nodes = np.array([[0.0, 0.0, 0.0], [h, 0.0, 0.0], [h / 2, h * math.sqrt(3) / 2, 0.0]])
    g = element_geometry(nodes, np.array([[0, 1, 2]]))
    assert g["A"][0] == pytest.approx(math.sqrt(3) * h * h / 4, rel=1e-14)


@pytest.mark.parametrize("subdiv", [1, 2, 3])
def test_icosphere_normals_unit_and_outward(subdiv):
    nodes, tris = synth.icosphere(subdiv)
    g = element_geometry(nodes, tris)
    assert np.allclose(np.linalg.norm(g["n"], axis=1), 1.0, atol=1e-14)
    # outward: the normal points away from the centre of the sphere; the
    # collocation point lies just inside the unit sphere (vertices on it)
    radial = g["x"] / np.linalg.norm(g["x"], axis=1, keepdims=True)
    assert np.min(np.sum(g["n"] * radial, axis=1)) > 0.95
    assert np.max(np.linalg.norm(g["x"], axis=1)) < 1.0


def test_icosphere_area_converges_to_sphere_at_second_order():
    # inscribed polyhedra: total area below 4 pi, the gap shrinking like h^2
    # (a factor 4 per subdivision, which halves the edge length)
    gaps = []
    for s in range(1, 6):
        nodes, tris = synth.icosphere(s)
        area = float(np.sum(element_geometry(nodes, tris)["A"]))
        assert area < 4 * math.pi
        gaps.append(4 * math.pi - area)
    ratios = [gaps[i] / gaps[i + 1] for i in range(len(gaps) - 1)]
    assert all(3.6 < r < 4.4 for r in ratios[1:]), ratios
    assert gaps[-1] < 2e-3 * 4 * math.pi
