"""Frequency sweep (paper_2312_00005_amd.sweep): per-frequency choice of the
far-field method and the solves it schedules.

1280-triangle sphere, leaf clusters of ~16 elements, candidate depths 3 and 2,
100-600 Hz in air: the two lowest frequencies have k X_min too small for the
expansion (stability cap) and run the direct far field, the others the FMM.
Checks: the choice; direct-far-field solutions against the oracle's LU
solution with the same rules (1e-9); FMM solutions through their residual in
dense oracle rows with converged quadrature (1e-6, the expansion accuracy);
every solve converged to the requested 1e-10."""

import math

import numpy as np
import pytest

import synth
from oracle import operator as op
from oracle.geometry import element_geometry
from oracle.presets import preset
from gpu_util import to_host, rel_l2, announce

pytestmark = pytest.mark.gpu

FREQS = [100.0, 200.0, 400.0, 600.0]


def test_sweep_methods_and_solutions():
    from paper_2312_00005_amd import sweep
    announce("sweep ico3 leaf 16, 4 frequencies, one stream")
    nodes, tris = synth.icosphere(3)
    g = element_geometry(nodes, tris)
    S = sweep.FrequencySweep(nodes, tris, FREQS, preset="mixed", depths=(3, 2), leaf_size=16, streams=1,
                             gmres_tol=1e-10)
    assert [m[0] for m in S.methods] == ["direct", "direct", "fmm", "fmm"]
    results, tot = S.run()
    announce(f"  totals {tot}")
    p_mixed = preset("mixed")
    rows = np.random.default_rng(3).choice(len(tris), 64, replace=False)
    for r in results:
        k = r["k"]
        p = to_host(r["p"])
        assert r["info"]["rel_residual"] < 1e-10
        b = op.rhs_plane_wave(g, k, (0.0, 0.0, 1.0), p=p_mixed)
        if r["method"][0] == "direct":
            ref = op.lu_solve(op.dense(g, k, p=p_mixed), b)
            err = rel_l2(p, ref)
        else:
            Ar = op.rows(g, rows, k, p=preset("mixed", quad_eps=1e-11))
            err = np.linalg.norm(b[rows] - Ar @ p) / np.linalg.norm(b[rows])
        announce(f"  f={r['f']:.0f} k={k:.2f} {r['method']} it={r['info']['iterations']} err={err:.2e}")
        assert err < (1e-9 if r["method"][0] == "direct" else 1e-6)


@pytest.mark.skip(reason="two host threads solving concurrently (two streams) ended once in a host "
                         "segmentation fault inside bem_solve; the cause is not found, so the mode is "
                         "disabled in the sweep and stays off the GPU")
def test_sweep_two_streams():
    from paper_2312_00005_amd import sweep
    nodes, tris = synth.icosphere(3)
    sweep.FrequencySweep(nodes, tris, FREQS, preset="mixed", depths=(3, 2), leaf_size=16, streams=2)


def test_sweep_rejects_concurrent_streams():
    from paper_2312_00005_amd import sweep
    nodes, tris = synth.icosphere(2)
    with pytest.raises(NotImplementedError):
        sweep.FrequencySweep(nodes, tris, FREQS, preset="mixed", depths=(2,), leaf_size=16, streams=2)
