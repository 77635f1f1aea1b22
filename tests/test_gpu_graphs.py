"""Captured operator applications (use_graphs = 1) replay the same kernels as
the eager path: GMRES solves with and without graphs agree bit for bit
(every kernel is deterministic), for the FMM and the direct far field, A and
A^H, FP64 and mixed precision, across a change of wavenumber (which forces a
new capture) and with eager Krylov work between the replays.  Eager FMM
applications also run the leaf-level translation on a third stream, which
captured ones do not, so the comparison covers that split as well."""

import math

import numpy as np
import pytest

import synth
from gpu_util import to_dev, to_host, announce

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bem():
    from paper_2312_00005_amd import bemfmm
    return bemfmm


@pytest.mark.parametrize("far_direct", [0, 1])
@pytest.mark.parametrize("pre", ["tight", "mixed"])
def test_graph_solves_match_eager(bem, far_direct, pre):
    announce(f"graphs vs eager ico4 {pre} far_direct={far_direct}")
    nodes, tris = synth.icosphere(4)
    h = synth.mean_edge_length(nodes, tris)
    kw = dict(use_fmm=1, levels=3, leaf_size=32, far_direct=far_direct, gmres_tol=1e-9)
    meshes = {g: bem.Mesh(nodes, tris, pre, use_graphs=g, **kw) for g in (0, 1)}
    rhs2 = to_dev(synth.complex_normal(len(tris), seed=8))
    for epw in (6.0, 10.0):
        k = 2 * math.pi / (epw * h)
        out = {}
        for g, m in meshes.items():
            m.set_problem(k)
            p, _, info = m.solve(m.rhs_plane_wave((0.0, 0.0, 1.0)))
            x, info_h = m.solve_adjoint(rhs2)
            out[g] = (to_host(p), info["iterations"], to_host(x), info_h["iterations"])
        announce(f"  k={k:.2f} iterations {out[1][1]} / {out[1][3]}")
        assert out[0][1] == out[1][1] and out[0][3] == out[1][3]
        assert np.array_equal(out[0][0], out[1][0])
        assert np.array_equal(out[0][2], out[1][2])


def test_autotune_keeps_results(bem):
    """Every launch shape the tuner may pick gives bit-identical operator
    applications (one owner per output, fixed summation order)."""
    announce("autotune ico5 tight")
    nodes, tris = synth.icosphere(5)
    k = 2 * math.pi / (6.0 * synth.mean_edge_length(nodes, tris))
    m = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32)
    m.set_problem(k)
    x = to_dev(synth.complex_normal(len(tris), seed=4))
    before = {p: to_host(m.apply(x, prec=p)) for p in ("fp64", "mixed")}
    picks = m.autotune()
    announce(f"  picks {picks}")
    assert set(picks["near_wpb"].values()) <= {1, 2, 4, 8}
    assert {t & ~(4096 | 8192) for t in picks["translate_tpb"].values()} <= {64, 128, 256}
    assert set(picks["near_waves_per_cu"].values()) <= {0, 8, 12, 16, 24}
    assert set(picks["near_split"].values()) <= {50, 60, 70, 80, 90, 100}
    for p in ("fp64", "mixed"):
        assert np.array_equal(to_host(m.apply(x, prec=p)), before[p])
    # a resident near-field grid (each wavefront looping over targets) changes
    # no output either
    m8 = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32, near_waves_per_cu=8)
    m8.set_problem(k)
    for p in ("fp64", "mixed"):
        assert np.array_equal(to_host(m8.apply(x, prec=p)), before[p])
    # nor does splitting the near field around the far field
    for split in (50, 80):
        ms = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32, near_waves_per_cu=8, near_split=split)
        ms.set_problem(k)
        for p in ("fp64", "mixed"):
            assert np.array_equal(to_host(ms.apply(x, prec=p)), before[p])
        ms.close()
    # nor do the translation blocks in XCD slab or node-range order
    for shape in (4096 + 64, 4096 + 256, 8192 + 64, 8192 + 128, 8192 + 256):
        ms = bem.Mesh(nodes, tris, "tight", use_fmm=1, levels=3, leaf_size=32, translate_shape=shape)
        ms.set_problem(k)
        for p in ("fp64", "mixed"):
            assert np.array_equal(to_host(ms.apply(x, prec=p)), before[p])
            assert np.array_equal(to_host(ms.apply(x, op="AH", prec=p)), to_host(m.apply(x, op="AH", prec=p)))
        ms.close()
    p1, _, info = m.solve(m.rhs_plane_wave((0.0, 0.0, 1.0)))
    assert info["rel_residual"] < 1e-6
