"""Prescribed normal velocities (VELO, alone and with ADMI) through
bem_rhs_velocity: the right-hand-side term and the solution against the
oracle's dense operators (1280 triangles, every pair by the near-field
kernels), and a pulsating sphere at 20480 triangles with the FMM against its
analytic surface pressure rho c u (i k a)/(i k a - 1)."""

import math

import numpy as np
import pytest

import synth
from oracle import operator as op
from oracle import velocity as ovel
from oracle.geometry import element_geometry
from oracle.presets import preset
from gpu_util import to_dev, to_host, rel_l2, announce

pytestmark = pytest.mark.gpu

RHO_C = 1.21 * 343.0


@pytest.fixture(scope="module")
def bem():
    from paper_2312_00005_amd import bemfmm
    return bemfmm


def test_velocity_rhs_and_solution_match_oracle(bem):
    announce("VELO + ADMI ico3 tight, all pairs near")
    nodes, tris = synth.icosphere(3)
    g = element_geometry(nodes, tris)
    N = len(tris)
    k = 2.0
    rng = np.random.default_rng(11)
    u = np.where(g["x"][:, 2] > 0.3, 1e-3 * (rng.normal(size=N) + 1j * rng.normal(size=N)), 0.0)
    beta = np.where(g["x"][:, 0] > 0.0, 0.4 - 0.2j, 0.0).astype(np.complex128)
    m = bem.Mesh(nodes, tris, "tight", use_fmm=0, gmres_tol=1e-12)
    m.set_problem(k, to_dev(beta))
    rhs = m.rhs_plane_wave((0.0, 0.0, 1.0))
    rhs = m.rhs_add_velocity(rhs, to_dev(u), RHO_C)
    pt = preset("tight")
    b = op.rhs_plane_wave(g, k, (0.0, 0.0, 1.0), p=pt) + ovel.velocity_rhs(g, k, u, RHO_C, p=pt)
    e_rhs = rel_l2(to_host(rhs), b)
    p, _, info = m.solve(rhs)
    ref = op.lu_solve(op.dense(g, k, beta=beta, p=pt), b)
    e_p = rel_l2(to_host(p), ref)
    announce(f"  rhs {e_rhs:.2e}  solution {e_p:.2e}  iterations {info['iterations']}")
    assert e_rhs < 1e-11
    assert e_p < 1e-9


def test_pulsating_sphere_with_fmm(bem):
    announce("pulsating sphere ico5 tight, 3-level FMM")
    nodes, tris = synth.icosphere(5)
    N = len(tris)
    k = 2.0
    u0 = 1e-3
    m = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32, gmres_tol=1e-8)
    m.set_problem(k)
    rhs = m.rhs_add_velocity(to_dev(np.zeros(N, dtype=np.complex128)), to_dev(np.full(N, u0 + 0j)), RHO_C)
    p, _, info = m.solve(rhs)
    exact = RHO_C * u0 * (1j * k) / (1j * k - 1.0)
    err = np.max(np.abs(to_host(p) - exact)) / abs(exact)
    announce(f"  max rel. error {err:.2e} (first order in h), iterations {info['iterations']}")
    assert err < 0.01
    with pytest.raises(bem.BemError) as e:
        m.rhs_add_velocity(rhs, to_dev(np.zeros(N, dtype=np.complex128)), -1.0)
    assert e.value.status == bem.BEM_E_ARG
