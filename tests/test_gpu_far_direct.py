"""GPU parity of the direct far field (far_direct = 1): the cluster tree and
near plan are kept, every admissible pair is integrated on the fly with the
rule the near plan would choose.  The whole operator is then the dense
operator itself, so it is compared with the oracle's dense matrix entry for
entry through matvecs: FP64 to 1e-12, complex FP32 to 2e-5 (relative to
max|y|), A^H and dA/dc likewise.  A 2/sqrt(3) tree (the paper's
admissibility) puts far pairs close enough to need subdivision."""

import numpy as np
import pytest

import synth
from oracle import adjoint as oadj
from oracle import operator as op
from oracle.geometry import element_geometry
from oracle.presets import preset
from gpu_util import to_dev, to_host, rel_max, announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bem():
    from paper_2312_00005_amd import bemfmm
    return bemfmm


CASES = [("paper", 2.0 / 3 ** 0.5, 2, 32, 3.0, True), ("tight", 3.0, 3, 8, 7.0, False),
         ("tight", 3.0, 2, 16, 2.0, True)]


@pytest.mark.parametrize("pre,adm,levels,leaf,k,with_beta", CASES)
def test_far_direct_is_the_dense_operator(bem, pre, adm, levels, leaf, k, with_beta):
    announce(f"far direct ico3 {pre} adm={adm:.3f} levels={levels} leaf={leaf} k={k} beta={with_beta}")
    nodes, tris = synth.icosphere(3)
    g = element_geometry(nodes, tris)
    N = len(tris)
    beta = (1.0 + 0.5 * synth.uniform01(N, seed=1)) + 0.3j if with_beta else None
    p = preset(pre, admissibility=adm)
    A = op.dense(g, k, beta=beta, p=p)
    m = bem.Mesh(nodes, tris, pre, use_fmm=1, levels=levels, leaf_size=leaf, admissibility=adm, far_direct=1)
    m.set_problem(k, None if beta is None else to_dev(beta))
    far_pairs = N * N - m.stats()["near_pairs"]
    announce(f"  far pairs {far_pairs} of {N * N}")
    assert far_pairs > N * N // 5
    x = synth.complex_normal(N, seed=4)
    xd = to_dev(x)
    assert rel_max(to_host(m.apply(xd)), A @ x) < 1e-12
    assert rel_max(to_host(m.apply(xd, op="AH")), A.conj().T @ x) < 1e-12
    assert rel_max(to_host(m.apply(xd, prec="mixed")), A @ x) < 2e-5
    assert rel_max(to_host(m.apply(xd, op="AH", prec="mixed")), A.conj().T @ x) < 2e-5
    if with_beta:
        V = oadj.dense_dc(g, k, p)
        assert rel_max(to_host(m.apply_dc(xd)), V @ x) < 1e-12
        assert rel_max(to_host(m.apply_dc(xd, op="AH")), V.conj().T @ x) < 1e-12


def test_far_direct_solve_matches_lu(bem):
    announce("far direct solve ico3 tight k=4")
    nodes, tris = synth.icosphere(3)
    g = element_geometry(nodes, tris)
    k = 4.0
    A = op.dense(g, k, p=preset("tight"))
    b = op.rhs_plane_wave(g, k, (0.0, 0.0, 1.0), p=preset("tight"))
    m = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=8, far_direct=1, gmres_tol=1e-12)
    m.set_problem(k)
    p, _, info = m.solve(m.rhs_plane_wave((0.0, 0.0, 1.0)))
    assert info["rel_residual"] < 1e-12
    assert rel_max(to_host(p), op.lu_solve(A, b)) < 1e-10


@pytest.mark.parametrize("pre,adm,levels,leaf,k,with_beta", CASES)
def test_far_rows_match_one_point_per_wavefront(bem, pre, adm, levels, leaf, k, with_beta):
    """The forward direct far field with four collocation points of a leaf
    per wavefront (far_rows = 4, the default) sums every point's pairs in the
    order of the one-point-per-wavefront kernel; the compiler may contract
    the two kernels' arithmetic differently, so they agree to rounding:
    1e-13 (FP64) and 1e-6 (complex FP32) relative to max|y|, with admittance
    and for dA/dc."""
    announce(f"far rows ico3 {pre} adm={adm:.3f} levels={levels} leaf={leaf} k={k} beta={with_beta}")
    nodes, tris = synth.icosphere(3)
    N = len(tris)
    beta = (1.0 + 0.5 * synth.uniform01(N, seed=1)) + 0.3j if with_beta else None
    meshes = [bem.Mesh(nodes, tris, pre, use_fmm=1, levels=levels, leaf_size=leaf, admissibility=adm, far_direct=1,
                       far_rows=r) for r in (1, 4)]
    for m in meshes:
        m.set_problem(k, None if beta is None else to_dev(beta))
    xd = to_dev(synth.complex_normal(N, seed=4))
    for prec, tol in (("fp64", 1e-13), ("mixed", 1e-6)):
        a, b = (to_host(m.apply_part(xd, 2, prec=prec)) for m in meshes)
        e = rel_max(b, a)
        announce(f"  {prec}: far_rows 4 vs 1 {e:.1e}")
        assert e < tol
    if with_beta:
        a, b = (to_host(m.apply_dc(xd)) for m in meshes)
        assert rel_max(b, a) < 1e-13
    for m in meshes:
        m.close()
