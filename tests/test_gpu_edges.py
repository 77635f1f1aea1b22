"""Edge cases of the C ABI on the GPU: a one-element mesh, a zero right-hand
side, field points on the surface (a bounded subdivision that ends in
BEM_E_MESH), empty point sets, calls before bem_set_problem and invalid
wavenumbers.  Every case ends with a status code; none relies on a fault."""

import math

import numpy as np
import pytest

import synth
from oracle import operator as op
from oracle.geometry import element_geometry
from oracle.presets import preset
from gpu_util import to_dev, to_host, rel_max, announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bem():
    from paper_2312_00005_amd import bemfmm
    return bemfmm


def test_single_element(bem):
    announce("single element")
    nodes = np.array([[0.0, 0.0, 0.0], [0.3, 0.0, 0.0], [0.0, 0.4, 0.0]])
    tris = np.array([[0, 1, 2]], dtype=np.int32)
    g = element_geometry(nodes, tris)
    k = 2.0
    A = op.dense(g, k, p=preset("paper"))
    m = bem.Mesh(nodes, tris, "paper", use_fmm=0)
    m.set_problem(k)
    x = np.array([1.0 - 0.5j])
    assert rel_max(to_host(m.apply(to_dev(x))), A @ x) < 1e-13
    b = op.rhs_plane_wave(g, k, (0.0, 0.0, 1.0))
    p, _, info = m.solve(m.rhs_plane_wave((0.0, 0.0, 1.0)))
    assert rel_max(to_host(p), b / A[0, 0]) < 1e-12


def test_zero_rhs_gives_zero(bem):
    announce("zero rhs")
    nodes, tris = synth.icosphere(2)
    for pre, kw in (("paper", dict(use_fmm=0)), ("mixed", dict(use_fmm=1, levels=2, leaf_size=32))):
        m = bem.Mesh(nodes, tris, pre, **kw)
        m.set_problem(1.5)
        z = to_dev(np.zeros(len(tris), dtype=np.complex128))
        p, _, info = m.solve(z)
        assert info["iterations"] == 0
        assert np.all(to_host(p) == 0)
        x, info_h = m.solve_adjoint(z)
        assert np.all(to_host(x) == 0)


def test_field_points_on_the_surface_are_a_mesh_error(bem):
    import torch
    announce("field point on the surface")
    nodes, tris = synth.icosphere(2)
    g = element_geometry(nodes, tris)
    m = bem.Mesh(nodes, tris, "paper", use_fmm=0)
    m.set_problem(2.0)
    p = to_dev(synth.complex_normal(len(tris), seed=1))
    pts = torch.from_numpy(np.array([[0.0, 0.0, 2.0], g["x"][7]])).to("cuda")
    with pytest.raises(bem.BemError) as e:
        m.field(pts, p)
    assert e.value.status == bem.BEM_E_MESH
    # no points: nothing to do
    empty = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    assert m.field(empty, p).numel() == 0


def test_calls_before_set_problem_and_bad_wavenumbers(bem):
    announce("state and argument errors")
    nodes, tris = synth.icosphere(1)
    m = bem.Mesh(nodes, tris, "paper", use_fmm=0)
    x = to_dev(np.ones(len(tris), dtype=np.complex128))
    with pytest.raises(bem.BemError) as e:
        m.apply(x)
    assert e.value.status == bem.BEM_E_STATE
    with pytest.raises(bem.BemError) as e:
        m.solve(x)
    assert e.value.status == bem.BEM_E_STATE
    for k in (0.0, -1.0, math.nan, math.inf):
        with pytest.raises(bem.BemError) as e:
            m.set_problem(k)
        assert e.value.status == bem.BEM_E_ARG
    m.set_problem(1.0)
    assert np.all(np.isfinite(to_host(m.apply(x))))
