"""Full-size parity of the frequency sweep's workload (40500-triangle rigid
sphere, plane wave) at three of its 64 frequencies (100 Hz, ~1 kHz, ~2.1 kHz)
against the CPU oracle's LU solutions stored in tests/golden/c4_sphere40500.npz
(written by tests/golden/make_c4_golden.py from oracle/ alone, converged
quadrature).  The sweep chooses the far-field method per frequency as in its
timed runs (direct far field where the expansion is not stable, FMM
otherwise); surface pressure within 1e-5 (FP64 GMRES) and 1e-3 (mixed
precision) of the LU solution (relative l2)."""

import os

import numpy as np
import pytest

import synth
from gpu_util import to_host, rel_l2, announce

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c4_sphere40500.npz")


@pytest.mark.parametrize("prec,tol,gate", [("fp64", 1e-9, 1e-5), ("mixed", 1e-7, 1e-3)])
def test_c4_sweep_pressure_vs_lu(prec, tol, gate):
    if not os.path.exists(GOLDEN):
        pytest.skip("c4 golden file not generated (tests/golden/make_c4_golden.py)")
    from paper_2312_00005_amd.sweep import FrequencySweep
    z = np.load(GOLDEN)
    nodes, tris = synth.geodesic_sphere(45)
    idx = [int(i) for i in z["indices"]]
    freqs = [100.0 * 200.0 ** (i / 63.0) for i in idx]
    announce(f"c4 sweep vs oracle LU at {[round(f, 1) for f in freqs]} Hz, {prec}")
    sw = FrequencySweep(nodes, tris, freqs, c=float(z["c"]), preset="tight" if prec == "fp64" else "mixed",
                        gmres_tol=tol)
    res, tot = sw.run()
    for r, i in zip(res, idx):
        assert abs(r["k"] - float(z[f"k_{i}"])) < 1e-12 * r["k"]
        p = to_host(r["p"])
        e = rel_l2(p, z[f"p_lu_{i}"])
        emax = np.max(np.abs(p - z[f"p_lu_{i}"])) / np.max(np.abs(z[f"p_lu_{i}"]))
        announce(f"  f = {r['f']:.1f} Hz, {r['method']}, {r['info']['iterations']} iterations: "
                 f"rel l2 {e:.2e}, max {emax:.2e}")
        assert e < gate
