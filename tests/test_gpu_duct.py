"""The duct of Sec. 5.3 on the GPU: interior problem (tau = -1), normal
velocity 1 m/s at x = 0, admittance 1/(rho c) at x = L = 3.4 m, sound-hard
sides of the 0.2 x 0.2 m cross section; closed-form solution
p(x) = -rho c exp(ikx) (Eq. (PlaneWaveSol)).

* 1260 triangles, every pair by the near-field kernels: the surface pressure
  equals the oracle's LU solution of the same system (1e-9), and the
  pressure at points inside the duct (bem_field_pv with the interior sign)
  equals the oracle's representation formula (1e-12).
* 8960 triangles (edge 0.025 m, one of the paper's two meshes): the 3-level
  FMM at 480 Hz and the direct far field at 240 Hz (where the expansion's
  stability cap would bind) against the all-pairs operator (1e-6) and, as
  solutions, against the plane wave within the paper's 6 %."""

import math

import numpy as np
import pytest

import synth
from oracle import field, operator as op, velocity
from oracle.geometry import element_geometry
from oracle.presets import preset
from gpu_util import to_dev, to_host, rel_l2, announce

pytestmark = pytest.mark.gpu

RHO, C = 1.3, 340.0
LENGTH = 3.4


@pytest.fixture(scope="module")
def bem():
    from paper_2312_00005_amd import bemfmm
    return bemfmm


def _duct(h):
    nodes, tris = synth.box((LENGTH, 0.2, 0.2), h, origin=(0.0, -0.1, -0.1))
    g = element_geometry(nodes, tris)
    x = g["x"][:, 0]
    u = np.where(x < 1e-9, 1.0 + 0j, 0.0)
    beta = np.where(x > LENGTH - 1e-9, 1.0 + 0j, 0.0)
    return nodes, tris, g, u, beta


def _solve(bem, mesh, k, u, beta):
    mesh.set_problem(k, to_dev(beta))
    rhs = to_dev(np.zeros(len(u), dtype=np.complex128))
    mesh.rhs_add_velocity(rhs, to_dev(u), RHO * C)
    p, _, info = mesh.solve(rhs)
    return to_host(p), info


@pytest.mark.parametrize("f", [240.0, 480.0])
def test_duct_matches_oracle(bem, f):
    import torch
    announce(f"duct 1260 triangles, {f} Hz, all pairs direct")
    nodes, tris, g, u, beta = _duct(0.2 / 3)
    k = 2 * math.pi * f / C
    rc = RHO * C
    m = bem.Mesh(nodes, tris, "tight", use_fmm=0, interior=1, gmres_tol=1e-12, gmres_maxit=1000)
    p, info = _solve(bem, m, k, u, beta)
    pt = preset("tight")
    A = op.dense(g, k, beta=beta, p=pt, tau=-1)
    ref = op.lu_solve(A, velocity.velocity_rhs(g, k, u, rc, p=pt, tau=-1))
    e = rel_l2(p, ref)
    ex = -rc * np.exp(1j * k * g["x"][:, 0])
    announce(f"  vs oracle LU {e:.1e} ({info['iterations']} iterations), vs plane wave {rel_l2(p, ex):.3f}")
    assert e < 1e-9
    v = op.bc_factor(k, beta, tau=-1) * p + 1j * k * rc * u
    pts = np.stack([np.linspace(0.3, 3.1, 8), np.zeros(8), np.zeros(8)], axis=1)
    ptsd = torch.from_numpy(pts).to("cuda")
    inside = to_host(m.field_pv(ptsd, to_dev(p), to_dev(v)))
    ref_in = field.field_pv(g, pts, k, p, v, p=pt, tau=-1)
    assert rel_l2(inside, ref_in) < 1e-12
    assert np.max(np.abs(inside + rc * np.exp(1j * k * pts[:, 0]))) / rc < 0.2


@pytest.mark.parametrize("f,far_direct", [(480.0, 0), (240.0, 1)])
def test_duct_paper_mesh_with_tree(bem, f, far_direct):
    announce(f"duct 8960 triangles, {f} Hz, 3-level tree, far_direct={far_direct}")
    nodes, tris, g, u, beta = _duct(0.025)
    k = 2 * math.pi * f / C
    rc = RHO * C
    mt = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32, interior=1, far_direct=far_direct,
                  gmres_tol=1e-8, gmres_maxit=1000)
    md = bem.Mesh(nodes, tris, "tight", use_fmm=0, interior=1)
    mt.set_problem(k, to_dev(beta))
    md.set_problem(k, to_dev(beta))
    x = to_dev(synth.complex_normal(len(tris), seed=4))
    e_op = rel_l2(to_host(mt.apply(x)), to_host(md.apply(x)))
    p, info = _solve(bem, mt, k, u, beta)
    ex = -rc * np.exp(1j * k * g["x"][:, 0])
    e = rel_l2(p, ex)
    announce(f"  operator vs all pairs {e_op:.1e}; solution vs plane wave {e:.3f} ({info['iterations']} iterations)")
    assert e_op < 1e-6
    assert e < 0.06
