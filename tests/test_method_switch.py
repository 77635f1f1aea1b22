"""The paper's automatic change of method (Sec. 3.3.4, Fig. FMMChange),
host logic of the library (bem_auto_method, bem_mesh_diameter): each rule of
the text at and around its threshold, and the diameter of meshes whose
largest node distance is known in closed form."""

import math

import numpy as np
import pytest

import synth

BEM, SL, ML = 0, 1, 4


@pytest.fixture(scope="module")
def bem():
    from paper_2312_00005_amd import bemfmm
    return bemfmm


def lam(k):
    return 2 * math.pi / k


def k_for(wavelength):
    return 2 * math.pi / wavelength


@pytest.mark.parametrize("req,n,wl_over_d,expect", [
    # conventional BEM asked for: more than 20000 elements -> SLFMM, more than 50000 -> MLFMM
    (BEM, 20000, 0.5, BEM), (BEM, 20001, 0.5, SL), (BEM, 50000, 0.5, SL), (BEM, 50001, 0.5, ML),
    # SLFMM asked for: more than 50000 -> MLFMM
    (SL, 50000, 0.5, SL), (SL, 50001, 0.5, ML),
    # an FMM at a wavelength of 80 diameters or more -> conventional BEM
    (ML, 30000, 80.0, BEM), (SL, 30000, 80.0, BEM), (ML, 30000, 79.0, SL), (SL, 30000, 79.0, SL),
    # MLFMM at a wavelength above the diameter -> SLFMM; at or below it stays
    (ML, 30000, 1.01, SL), (ML, 30000, 1.0, ML), (ML, 30000, 0.3, ML),
    # the upgrades come first: BEM asked for on a large mesh at a long wavelength
    (BEM, 60000, 100.0, BEM), (BEM, 60000, 2.0, SL), (BEM, 60000, 0.5, ML),
])
def test_switch_rules(bem, req, n, wl_over_d, expect):
    D = 1.7
    # the wavelength exactly wl_over_d diameters (k from it), up to rounding
    k = k_for(wl_over_d * D)
    if wl_over_d == 1.0:
        k *= 1.0 + 1e-12  # strictly not longer than the diameter
    if wl_over_d == 80.0:
        k *= 1.0 - 1e-12  # at least 80 diameters
    assert bem.bem_auto_method(req, n, D, k) == expect


def test_switch_argument_errors(bem):
    with pytest.raises(bem.BemError):
        bem.bem_auto_method(2, 100, 1.0, 1.0)
    with pytest.raises(bem.BemError):
        bem.bem_auto_method(BEM, 100, 0.0, 1.0)


def test_mesh_diameter(bem):
    # the icosahedron's vertices come in antipodal pairs, and so do those of
    # its refinements projected to the sphere: diameter 2 r
    nodes, _ = synth.icosphere(3, radius=1.5)
    assert bem.bem_mesh_diameter(nodes) == pytest.approx(3.0, rel=1e-14)
    # box: the space diagonal
    nodes, _ = synth.box((3.4, 0.2, 0.2), 0.1)
    assert bem.bem_mesh_diameter(nodes) == pytest.approx(math.sqrt(3.4 ** 2 + 0.08), rel=1e-14)
    # brute force on a random cloud
    pts = np.random.default_rng(3).standard_normal((300, 3))
    d = np.sqrt(((pts[:, None, :] - pts[None, :, :]) ** 2).sum(-1)).max()
    assert bem.bem_mesh_diameter(pts) == pytest.approx(d, rel=1e-15)
