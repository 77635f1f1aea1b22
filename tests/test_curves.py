"""The library's frequency and admittance curves (host side) against the
oracle's, and the sweep's refusal of an admittance without frequency steps."""

import numpy as np
import pytest

from oracle import curves as oc
from paper_2312_00005_amd import curves


def test_curve_matches_oracle_on_random_curves():
    rng = np.random.default_rng(3)
    for _ in range(100):
        n = int(rng.integers(2, 8))
        s = np.cumsum(rng.uniform(0.1, 2.0, n))
        v = rng.normal(size=n)
        nodes = list(zip(s.tolist(), v.tolist()))
        C = curves.Curve(nodes)
        for q in np.concatenate([s, rng.uniform(s[0], s[-1], 16)]):
            assert C(q) == pytest.approx(oc.curve_value(nodes, q), abs=1e-12)
        with pytest.raises(ValueError):
            C(s[-1] + 1e-9)


def test_steps_frequencies_and_groups():
    nodes = [(0.0, 35.481), (3.0, 44.668), (6.0, 56.234)]
    assert np.allclose(curves.frequencies(6, 1.0, 0.0, curves.Curve(nodes)), oc.frequencies(6, 1.0, 0.0, nodes))
    re_n, im_n = [(0.0, 0.0), (1.0, 1.0), (3.0, 4.0)], [(0.0, 0.0), (3.0, 2.0)]
    g1 = curves.AdmittanceGroup(np.array([0, 2]), 0.3 - 0.1j, curves.Curve(re_n), curves.Curve(im_n))
    g2 = curves.AdmittanceGroup(np.array([2, 3]), 1.0 + 1.0j)
    y = curves.element_admittance([g1, g2], 5, 2.5)
    assert y[0] == pytest.approx(oc.admittance(2.5, 0.3 - 0.1j, re_n, im_n))
    assert y[1] == 0 and y[4] == 0
    assert y[2] == y[3] == 1.0 + 1.0j  # the later group wins
    with pytest.raises(ValueError):
        curves.element_admittance([curves.AdmittanceGroup(np.array([5]), 1.0)], 5, 0.0)


def test_sweep_needs_steps_for_admittance():
    from paper_2312_00005_amd import sweep
    import synth
    nodes, tris = synth.icosphere(1)
    g = curves.AdmittanceGroup(np.array([0]), 1.0)
    with pytest.raises(ValueError):
        sweep.FrequencySweep(nodes, tris, [100.0, 200.0], admittance=[g])
