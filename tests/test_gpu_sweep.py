"""Frequency sweep (paper_2312_00005_amd.sweep): per-frequency choice of the
far-field method and the solves it schedules.

1280-triangle sphere, leaf clusters of ~16 elements, candidate depths 3 and 2,
100-600 Hz in air: the lowest frequency has k X_min too small for the FP64
expansion (stability cap), so its FP64 operator (the refinement residuals)
integrates the far field directly while the complex-FP32 inner operator
keeps the FMM ("fmm32"); the others use the FMM throughout.
Checks: the choice; solutions whose FP64 operator is direct against the
oracle's LU solution with the same rules (1e-9); FMM solutions through their residual in
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
    assert [m[0] for m in S.methods] == ["fmm32", "fmm", "fmm", "fmm"]
    results, tot = S.run()
    announce(f"  totals {tot}")
    p_mixed = preset("mixed")
    rows = np.random.default_rng(3).choice(len(tris), 64, replace=False)
    for r in results:
        k = r["k"]
        p = to_host(r["p"])
        assert r["info"]["rel_residual"] < 1e-10
        b = op.rhs_plane_wave(g, k, (0.0, 0.0, 1.0), p=p_mixed)
        if r["method"][0] in ("direct", "fmm32"):
            ref = op.lu_solve(op.dense(g, k, p=p_mixed), b)
            err = rel_l2(p, ref)
        else:
            Ar = op.rows(g, rows, k, p=preset("mixed", quad_eps=1e-11))
            err = np.linalg.norm(b[rows] - Ar @ p) / np.linalg.norm(b[rows])
        announce(f"  f={r['f']:.0f} k={k:.2f} {r['method']} it={r['info']['iterations']} err={err:.2e}")
        assert err < (1e-9 if r["method"][0] in ("direct", "fmm32") else 1e-6)


def test_sweep_frequency_dependent_admittance():
    """Frequencies from a frequency-defining curve and an admittance whose real
    and imaginary parts follow two more curves of the frequency step, on the
    upper half of the sphere (input description, appendix): every solution
    against the oracle's LU solution with beta = rho c alpha(s) from the
    oracle's own curves."""
    from paper_2312_00005_amd import curves, sweep
    from oracle import curves as ocurves
    announce("sweep ico3 with admittance curves")
    nodes, tris = synth.icosphere(3)
    g = element_geometry(nodes, tris)
    upper = np.nonzero(g["x"][:, 2] > 0.0)[0]
    rho, c = 1.21, 343.0
    v0 = complex(0.5, -0.2) / (rho * c)
    fnodes = [(0.0, 0.0), (2.0, 200.0)]
    re_nodes, im_nodes = [(0.0, 0.5), (2.0, 1.5)], [(0.0, 1.0), (2.0, 2.0)]
    grp = curves.AdmittanceGroup(upper, v0, curves.Curve(re_nodes), curves.Curve(im_nodes))
    S = sweep.FrequencySweep.from_curve(nodes, tris, 2, 1.0, 0.0, curves.Curve(fnodes), c=c, rho=rho,
                                        preset="mixed", depths=(3, 2), leaf_size=16, admittance=[grp],
                                        gmres_tol=1e-10)
    assert S.freqs == pytest.approx(ocurves.frequencies(2, 1.0, 0.0, fnodes))
    results, _ = S.run()
    p_mixed = preset("mixed")
    for n, r in enumerate(results, start=1):
        s = ocurves.step_arguments(2, 1.0, 0.0)[n - 1]
        beta = np.zeros(len(tris), dtype=np.complex128)
        beta[upper] = rho * c * ocurves.admittance(s, v0, re_nodes, im_nodes)
        k = r["k"]
        b = op.rhs_plane_wave(g, k, (0.0, 0.0, 1.0), p=p_mixed)
        ref = op.lu_solve(op.dense(g, k, beta=beta, p=p_mixed), b)
        err = rel_l2(to_host(r["p"]), ref)
        announce(f"  step {n} f={r['f']:.0f} {r['method']} it={r['info']['iterations']} err={err:.2e}")
        # FP64 operator direct: the LU solution with the same rules; FMM: within
        # the expansion's accuracy
        assert err < (1e-9 if r["method"][0] in ("direct", "fmm32") else 1e-6)
    # the admittance changes the solution: against the sound-hard solve
    rigid = op.lu_solve(op.dense(g, results[-1]["k"], p=p_mixed),
                        op.rhs_plane_wave(g, results[-1]["k"], (0.0, 0.0, 1.0), p=p_mixed))
    assert rel_l2(to_host(results[-1]["p"]), rigid) > 1e-3


def test_sweep_source_strength_curves():
    """A plane wave whose strength follows curves of the frequency step: each
    solution is the constant-strength one times P0(s) (the operator is linear;
    GMRES is invariant to the scale of the right-hand side up to rounding)."""
    from paper_2312_00005_amd import curves, sweep
    from oracle import curves as ocurves
    announce("sweep ico3 with source-strength curves")
    nodes, tris = synth.icosphere(3)
    fn = curves.Curve([(0.0, 0.0), (2.0, 200.0)])
    re_nodes, im_nodes = [(0.0, 1.0), (2.0, 3.0)], [(0.0, 0.0), (2.0, -1.0)]
    S = sweep.FrequencySweep.from_curve(nodes, tris, 2, 1.0, 0.0, fn, preset="mixed", depths=(3, 2),
                                        leaf_size=16, gmres_tol=1e-11)
    P0 = complex(2.0, 0.5)
    src = ("plane", (0.0, 0.0, 1.0), P0)
    scaled, _ = S.run(source=src, source_curves=(curves.Curve(re_nodes), curves.Curve(im_nodes)))
    plain, _ = S.run(source=("plane", (0.0, 0.0, 1.0), 1.0))
    for n, (a, b) in enumerate(zip(scaled, plain), start=1):
        s = ocurves.step_arguments(2, 1.0, 0.0)[n - 1]
        strength = ocurves.admittance(s, P0, re_nodes, im_nodes)  # same scaling rule
        err = rel_l2(to_host(a["p"]), strength * to_host(b["p"]))
        announce(f"  step {n}: P0(s) = {strength:.3f}, err {err:.1e}")
        assert err < 1e-9


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


def test_sweep_paper_policy():
    """The paper's automatic switches (Sec. 3.3.4) as the sweep's method
    choice on the 1280-triangle unit sphere (diameter 2 m), multilevel FMM
    requested: 1 Hz (wavelength over 80 diameters) runs the conventional
    method and matches the oracle's LU solution to 1e-9; 100 Hz (wavelength
    above the diameter) the single-level FMM and 400 Hz the multilevel FMM,
    each within the paper's FMM-versus-direct difference of 1e-3 (Sec. 5.1.3)
    of the LU solution."""
    from paper_2312_00005_amd import sweep
    announce("sweep ico3, paper policy, 1 / 100 / 400 Hz")
    nodes, tris = synth.icosphere(3)
    g = element_geometry(nodes, tris)
    S = sweep.FrequencySweep(nodes, tris, [1.0, 100.0, 400.0], preset="mixed", depths=(2,), leaf_size=16,
                             policy="paper", gmres_tol=1e-10)
    assert S.methods == [("dense", 0), ("fmm", 1), ("fmm", 2)]
    results, _ = S.run()
    p_mixed = preset("mixed")
    for r in results:
        k = r["k"]
        b = op.rhs_plane_wave(g, k, (0.0, 0.0, 1.0), p=p_mixed)
        ref = op.lu_solve(op.dense(g, k, p=p_mixed), b)
        err = rel_l2(to_host(r["p"]), ref)
        announce(f"  f={r['f']:.0f} {r['method']} it={r['info']['iterations']} vs LU {err:.2e}")
        assert err < (1e-9 if r["method"][0] == "dense" else 1e-3)


def test_mesh_from_tree_equals_a_new_mesh():
    """A mesh made from a host tree (bem_mesh_create_from_tree: the tree's
    geometry, cluster tree and near plan, shared by the sweep's method groups
    of one depth) applies the same operator as a mesh built from the arrays,
    bit for bit, for each far-field method and both precisions."""
    from paper_2312_00005_amd import bemfmm
    import torch
    announce("mesh from a host tree vs a new mesh, ico3 depth 3")
    nodes, tris = synth.icosphere(3)
    t = bemfmm.HostTree(nodes, tris, "mixed", levels=3, leaf_size=16)
    x = torch.from_numpy(synth.complex_normal(len(tris), seed=4)).to("cuda")
    for far in (0, 1, 2):
        a = bemfmm.Mesh.from_tree(t, far_direct=far)
        b = bemfmm.Mesh(nodes, tris, "mixed", levels=3, leaf_size=16, far_direct=far)
        assert a.stats() == b.stats()
        for m in (a, b):
            m.set_problem(3.5)
        for prec in ("fp64", "mixed"):
            for o in ("A", "AH"):
                ya, yb = (to_host(m.apply(x, op=o, prec=prec)) for m in (a, b))
                assert np.array_equal(ya, yb), (far, prec, o)
        pa, _, ia = a.solve(a.rhs_plane_wave())
        pb, _, ib = b.solve(b.rhs_plane_wave())
        assert ia["iterations"] == ib["iterations"] and np.array_equal(to_host(pa), to_host(pb))
        a.close()
        b.close()


def test_probe_relabels_capped_frequencies():
    """Mixed path, GMRES tolerance 1e-6: the frequencies chosen as "fmm32"
    are probed on the device (capped FP64 FMM against the direct far field,
    relative l2 of A x); those at and above the lowest passing one take the
    FMM for their FP64 operator too.  Every probe that decided a relabelling
    passed at 1e-7, the relabelled set is the top of the group, and every
    solution is within 2e-5 of the oracle's LU solution with the same rules."""
    from paper_2312_00005_amd import sweep
    announce("sweep probe ico3 leaf 16, tol 1e-6")
    nodes, tris = synth.icosphere(3)
    g = element_geometry(nodes, tris)
    S = sweep.FrequencySweep(nodes, tris, FREQS, preset="mixed", depths=(3, 2), leaf_size=16, gmres_tol=1e-6)
    before = list(S.methods)
    results, tot = S.run()
    announce(f"  before {before}")
    announce(f"  after  {[r['method'] for r in results]}; probes {S.probes}; probe {tot['probe_s']:.2f} s")
    capped = [i for i, m in enumerate(before) if m[0] == "fmm32"]
    assert S.probes or not capped
    moved = [i for i in capped if results[i]["method"][0] == "fmm"]
    # the relabelled frequencies are the highest of the capped ones
    assert moved == capped[len(capped) - len(moved):]
    if moved:
        fmin = min(FREQS[i] for i in moved)
        assert any(p["pass"] and abs(p["f"] - fmin) < 1e-9 for p in S.probes)
    assert all(p["pass"] == (p["rel_l2"] <= 1e-7) for p in S.probes)
    p_mixed = preset("mixed")
    for r in results:
        k = r["k"]
        b = op.rhs_plane_wave(g, k, (0.0, 0.0, 1.0), p=p_mixed)
        ref = op.lu_solve(op.dense(g, k, p=p_mixed), b)
        err = rel_l2(to_host(r["p"]), ref)
        announce(f"  f={r['f']:.0f} {r['method']} it={r['info']['iterations']} vs LU {err:.2e}")
        assert r["info"]["rel_residual"] < 1e-6
        assert err < 2e-5
