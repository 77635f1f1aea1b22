"""GPU parity of the multilevel FMM far field and of the whole FMM operator.

* Same algorithm, same tree: the library's far-field part (bem_apply_part
  part 2) against the oracle's plain-steps FMM (oracle.fmm.FMM) on meshes that
  span several clusters per level, with and without resampling between
  levels.  FP64 to 1e-11 relative to max|y_far| (rounding; the library's Gauss
  nodes, Hankel recurrence and DFT factorisation differ from the oracle's
  only in rounding), or to ten times the rounding bound 2^-52 (2L+1)|h_L(k X_min)|
  where the translation operator amplifies rounding more; complex-FP32 to 3e-5.
* Whole operator: near field + far field against dense oracle rows whose
  quadrature is converged (tolerance 1e-11): the expansion is accurate to
  ~1e-8 there.  (Dense rows at the preset's own 1e-8 tolerance differ from
  the converged ones by ~1e-6 at 6 elements per wavelength: the a-priori
  order estimator of Sec. 3.1.4 does not see the oscillation of exp(ikr) on
  far elements, which the FMM's aggregation rule resolves.)
* Full-size workload (20480-triangle sphere, 3 levels, ~32 per leaf, 6
  elements per wavelength): sampled rows of the dense oracle, and the GMRES
  solution's residual in the oracle's operator at sampled rows."""

import math

import numpy as np
import pytest

import synth
from oracle import fmm as ofmm
from oracle import operator as op
from oracle import sphere
from oracle.geometry import element_geometry
from oracle.presets import preset
from gpu_util import to_dev, to_host, rel_max, rel_l2, announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bem():
    from paper_2312_00005_amd import bemfmm
    return bemfmm


def _k(nodes, tris, epw):
    return 2 * math.pi / (epw * synth.mean_edge_length(nodes, tris))


def _amplification(F, k):
    """Largest growth (2L+1)|h_L(k X_min)| of the translation operators."""
    amp = 1.0
    for Lv, L in zip(F.tree.levels, F.L):
        xm = ofmm.level_min_separation(Lv)
        if xm is not None:
            amp = max(amp, (2 * L + 1) * ofmm.hankel_abs(L, k * xm))
    return amp


FAR_CASES = [
    # mesh subdiv, levels, leaf, admissibility, preset, elements per wavelength, with beta
    (3, 2, 32, 2.0, "paper", 6.0, False),
    (4, 3, 32, 3.0, "tight", 20.0, True),   # L = 21/15/15: one level pair without resampling
    (4, 3, 32, 3.0, "tight", 6.0, False),
]


@pytest.mark.parametrize("subdiv,levels,leaf,adm,pre,epw,with_beta", FAR_CASES)
def test_far_field_matches_oracle_fmm(bem, subdiv, levels, leaf, adm, pre, epw, with_beta):
    announce(f"far field ico{subdiv} levels={levels} adm={adm} {pre} epw={epw} beta={with_beta}")
    nodes, tris = synth.icosphere(subdiv)
    g = element_geometry(nodes, tris)
    N = len(tris)
    k = _k(nodes, tris, epw)
    beta = None
    if with_beta:
        u = synth.uniform01(N, seed=1)
        beta = (1.0 + 0.5 * u) + 0.1j
    p = preset(pre, admissibility=adm)
    F = ofmm.FMM(g, k, p, levels, leaf, beta=beta)
    x = synth.complex_normal(N, seed=4)
    y_or = F.apply(x)
    m = bem.Mesh(nodes, tris, pre, use_fmm=1, levels=levels, leaf_size=leaf, admissibility=adm)
    m.set_problem(k, None if beta is None else to_dev(beta))
    xd = to_dev(x)
    y = to_host(m.apply_part(xd, 2))
    assert np.max(np.abs(y_or)) > 0
    # rounding differences are amplified by the translation operator's growth
    # (2L+1)|h_L(k X_min)| at small arguments: allow ten times that bound
    amp = _amplification(F, k)
    tol = max(1e-11, 10 * 2.2e-16 * amp)
    announce(f"  L={F.L} amplification={amp:.2e} tol={tol:.1e}")
    assert rel_max(y, y_or) < tol
    # complex-FP32 far field: its own truncation lengths (oracle single=True,
    # evaluated in FP64); FP32 rounding amplified by at most eps_mixed/10 by
    # construction of the lengths
    F32 = ofmm.FMM(g, k, p, levels, leaf, beta=beta, tree=F.tree, single=True)
    y_or32 = F32.apply(x)
    amp32 = _amplification(F32, k)
    tol32 = max(3e-5, 10 * 2.0 ** -23 * amp32)
    announce(f"  L32={F32.L} amplification={amp32:.2e} tol32={tol32:.1e}")
    y32 = to_host(m.apply_part(xd, 2, prec="mixed"))
    assert rel_max(y32, y_or32) < tol32
    # whole operator = dense rows restricted to near pairs + far field
    rows = np.random.default_rng(5).choice(N, 48, replace=False)
    Ar = op.rows(g, rows, k, beta=beta, p=p)
    mask = F.near_mask_rows(rows)
    y_full = to_host(m.apply(xd))
    ref = (Ar * mask) @ x + y_or[rows]
    assert rel_max(y_full[rows], ref) < tol
    if pre == "tight":
        # against the dense operator with converged quadrature
        Aref = op.rows(g, rows, k, beta=beta, p=preset(pre, admissibility=adm, quad_eps=1e-11))
        err = rel_l2(y_full[rows], Aref @ x)
        announce(f"  whole operator vs converged dense rows: {err:.2e}")
        assert err < 1e-6
    else:
        # the paper's preset against dense rows too: its far field (L from
        # Eq. (FMMTruncation) alone) against converged far entries, and the
        # whole operator against the converged dense operator, which differs
        # from it by the paper's own 1e-3 quadrature tolerance (Sec. 3.1.4)
        conv = preset(pre, admissibility=adm, quad_eps=1e-12, split_on_cap=True, self_n=12, edge_parts=8,
                      edge_gauss=6)
        Aref = op.rows(g, rows, k, beta=beta, p=conv)
        far_ref = (Ar * mask) @ x + (Aref * ~mask) @ x
        e_far = rel_l2(y_full[rows], far_ref)
        e_all = rel_l2(y_full[rows], Aref @ x)
        announce(f"  far field vs converged far entries {e_far:.2e}, whole operator vs converged dense {e_all:.2e}")
        assert e_far < 1e-5
        assert e_all < 1e-3


def test_fmm_levels_reported(bem):
    nodes, tris = synth.icosphere(4)
    g = element_geometry(nodes, tris)
    k = _k(nodes, tris, 6.0)
    m = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32)
    m.set_problem(k)
    F = ofmm.FMM(g, k, preset("tight"), 3, 32)
    F32 = ofmm.FMM(g, k, preset("tight"), 3, 32, tree=F.tree, single=True)
    rhs = m.rhs_plane_wave((0.0, 0.0, 1.0))
    p, _, info = m.solve(rhs)
    assert info["L"] == F.L
    assert info["L_mixed"] == F32.L
    assert info["clusters"] == [len(L["groups"]) for L in F.tree.levels]


@pytest.fixture(scope="module")
def c2(bem):
    nodes, tris = synth.icosphere(5)
    g = element_geometry(nodes, tris)
    k = _k(nodes, tris, 6.0)
    rows = np.random.default_rng(9).choice(len(tris), 24, replace=False)
    Ar = op.rows(g, rows, k, p=preset("tight", quad_eps=1e-11))
    return nodes, tris, g, k, rows, Ar


def test_full_size_operator_sampled_rows(bem, c2):
    announce("c2 operator sampled rows")
    nodes, tris, g, k, rows, Ar = c2
    m = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32)
    m.set_problem(k)
    x = synth.complex_normal(len(tris), seed=4)
    xd = to_dev(x)
    y = to_host(m.apply(xd))
    err = rel_l2(y[rows], Ar @ x)
    announce(f"  fp64 operator vs converged dense rows: {err:.2e}")
    assert err < 1e-7
    y32 = to_host(m.apply(xd, prec="mixed"))
    err32 = rel_l2(y32[rows], Ar @ x)
    announce(f"  fp32 operator vs converged dense rows: {err32:.2e}")
    assert err32 < 1e-4


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_full_size_solve(bem, c2, prec):
    announce(f"c2 solve {prec}")
    nodes, tris, g, k, rows, Ar = c2
    o = bem.bem_options_default("tight" if prec == "fp64" else "mixed")
    o.levels, o.leaf_size, o.gmres_tol = 3, 32, 1e-8
    m = bem.Mesh(nodes, tris, o)
    m.set_problem(k)
    rhs = m.rhs_plane_wave((0.0, 0.0, 1.0))
    p, _, info = m.solve(rhs)
    p = to_host(p)
    b = op.rhs_plane_wave(g, k, [0, 0, 1], p=preset("tight"))
    # residual of the GPU solution in the oracle's dense operator, sampled rows
    res = Ar @ p - b[rows]
    rr = np.linalg.norm(res) / np.linalg.norm(b[rows])
    announce(f"  residual in converged dense rows: {rr:.2e}, info {info}")
    assert rr < 1e-6
    assert info["rel_residual"] < 1e-8
    # discretisation-level agreement with the analytic rigid-sphere solution
    an = sphere.pressure(g["x"] / np.linalg.norm(g["x"], axis=1, keepdims=True), k)
    assert rel_l2(p, an) < 5e-2


@pytest.mark.parametrize("subdiv,levels,epw", [(4, 3, 6.0), (4, 3, 20.0), (3, 2, 6.0)])
def test_conjugate_transpose_dot_product(bem, subdiv, levels, epw):
    """<A x, y> = <x, A^H y> for the far field alone and for the whole
    operator, FP64 to 1e-12 (or ten times the translation operators' rounding
    amplification 2^-52 (2L+1)|h_L(k X_min)| where that is larger) and
    complex-FP32 to 1e-5 (the library's forward operator is itself pinned to
    the oracle above)."""
    announce(f"adjoint dot test ico{subdiv} levels={levels} epw={epw}")
    nodes, tris = synth.icosphere(subdiv)
    N = len(tris)
    k = _k(nodes, tris, epw)
    u = synth.uniform01(N, seed=1)
    beta = (1.0 + 0.5 * u) + 0.2j * u
    adm = 3.0 if subdiv == 4 else 2.0
    m = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=levels, leaf_size=32, admissibility=adm)
    m.set_problem(k, to_dev(beta))
    x = synth.complex_normal(N, seed=4)
    y = synth.complex_normal(N, seed=6)
    xd, yd = to_dev(x), to_dev(y)
    g = element_geometry(nodes, tris)
    amp = _amplification(ofmm.FMM(g, k, preset("tight", admissibility=adm), levels, 32, beta=beta), k)
    tol64 = max(1e-12, 10 * 2.2e-16 * amp)
    announce(f"  amplification={amp:.2e} tol64={tol64:.1e}")
    for prec, tol in (("fp64", tol64), ("mixed", 1e-5)):
        for part in (2, 0):
            Ax = to_host(m.apply_part(xd, part, prec=prec))
            AHy = to_host(m.apply_part(yd, part, op="AH", prec=prec))
            lhs = np.vdot(y, Ax)
            rhs = np.vdot(AHy, x)
            assert abs(lhs - rhs) < tol * np.linalg.norm(Ax) * np.linalg.norm(y), (prec, part, lhs, rhs)


@pytest.mark.parametrize("with_beta", [False, True])
def test_level_rows_far_field_matches_oracle(bem, with_beta):
    """The paper's level transfer (level_rows = 1: element-to-cluster rows on
    every level with interaction pairs) against the oracle's same variant,
    FP64 and complex FP32, its conjugate transpose by the dot-product
    identity, and the whole operator against the interpolating variant (both
    approximate the same far field to the expansion accuracy)."""
    announce(f"level rows ico4 levels=3 beta={with_beta}")
    nodes, tris = synth.icosphere(4)
    g = element_geometry(nodes, tris)
    N = len(tris)
    k = _k(nodes, tris, 6.0)
    beta = (1.0 + 0.5 * synth.uniform01(N, seed=1)) + 0.1j if with_beta else None
    p = preset("tight")
    F = ofmm.FMM(g, k, p, 3, 32, beta=beta, level_rows=True)
    assert sum(1 for L in F.tree.levels if any(len(il) for il in L["il"])) >= 2
    x = synth.complex_normal(N, seed=4)
    y_or = F.apply(x)
    m = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32, level_rows=1)
    m.set_problem(k, None if beta is None else to_dev(beta))
    xd = to_dev(x)
    amp = _amplification(F, k)
    tol = max(1e-11, 10 * 2.2e-16 * amp)
    assert rel_max(to_host(m.apply_part(xd, 2)), y_or) < tol
    F32 = ofmm.FMM(g, k, p, 3, 32, beta=beta, tree=F.tree, single=True, level_rows=True)
    tol32 = max(3e-5, 10 * 2.0 ** -23 * _amplification(F32, k))
    assert rel_max(to_host(m.apply_part(xd, 2, prec="mixed")), F32.apply(x)) < tol32
    yv = synth.complex_normal(N, seed=6)
    Ax = to_host(m.apply(xd))
    AHy = to_host(m.apply(to_dev(yv), op="AH"))
    assert abs(np.vdot(yv, Ax) - np.vdot(AHy, x)) < tol * np.linalg.norm(Ax) * np.linalg.norm(yv)
    mi = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32)
    mi.set_problem(k, None if beta is None else to_dev(beta))
    d = rel_l2(Ax, to_host(mi.apply(xd)))
    announce(f"  L={F.L} level rows vs interpolation: {d:.2e}")
    assert d < 1e-6
