"""Graded head-like workload: ellipsoid with semi-axes 0.075 x 0.09 x 0.11 m
and a raised bump on the +x side, ~60k triangles graded from ~0.7 mm edges on
the bump to ~5.7 mm elsewhere, point source 1 mm off the bump apex along its
normal, f = 16 kHz in air (c = 343 m/s), 5-level FMM, mixed precision.

The dense oracle does not fit (60500^2 complex entries), so parity uses
sampled rows: whole dense rows with converged quadrature (tolerance 1e-11) at
seeded collocation points, for the operator and for the residual of the GMRES
solution.  Tolerances: FP64 operator 1e-5 and mixed 1e-3 relative (the
accuracy targets of the two paths); the solution's residual in the oracle's
operator 2e-3 at the sampled rows (solver tolerance 1e-6 plus the mixed
operator's own error)."""

import math

import numpy as np
import pytest

import synth
from oracle import operator as op
from oracle.geometry import element_geometry
from oracle.presets import preset
from gpu_util import to_dev, to_host, rel_l2, announce

pytestmark = pytest.mark.gpu

K = 2 * math.pi * 16000.0 / 343.0


@pytest.fixture(scope="module")
def case():
    from paper_2312_00005_amd import bemfmm
    nodes, tris, apex, apex_n = synth.graded_ellipsoid_bump()
    announce(f"graded ellipsoid N={len(tris)} k={K:.3f}: building plan")
    m = bemfmm.Mesh(nodes, tris, "mixed", use_fmm=1, levels=5, leaf_size=32)
    m.set_problem(K, None)
    g = element_geometry(nodes, tris)
    rows = np.random.default_rng(5).choice(len(tris), 40, replace=False)
    Ar = op.rows(g, rows, K, p=preset("mixed", quad_eps=1e-11))
    src = apex + 1e-3 * apex_n
    return m, g, rows, Ar, src


def test_graded_operator_sampled_rows(case):
    m, g, rows, Ar, _ = case
    N = g["x"].shape[0]
    x = synth.complex_normal(N, seed=4)
    xd = to_dev(x)
    ref = Ar @ x
    e64 = rel_l2(to_host(m.apply(xd, prec="fp64"))[rows], ref)
    e32 = rel_l2(to_host(m.apply(xd, prec="mixed"))[rows], ref)
    announce(f"graded operator rows: fp64 {e64:.2e} mixed {e32:.2e} stats {m.stats()}")
    assert e64 < 1e-5
    assert e32 < 1e-3


def test_graded_point_source_solve(case):
    m, g, rows, Ar, src = case
    b = m.rhs_point_source(tuple(src), 1.0)
    bref = op.rhs_point_source(g, K, src, p=preset("mixed"))
    assert rel_l2(to_host(b), bref) < 1e-13
    p, _, info = m.solve(b)
    announce(f"graded solve: {info}")
    assert info["rel_residual"] < 1e-6
    ph = to_host(p)
    res = bref[rows] - Ar @ ph
    err = np.linalg.norm(res) / np.linalg.norm(bref[rows])
    announce(f"graded residual in the oracle's operator at sampled rows: {err:.2e}")
    assert err < 2e-3
