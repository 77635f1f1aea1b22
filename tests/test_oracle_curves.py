"""Pins of the oracle's frequency and admittance curves against the worked
examples the paper prints for its input description (tests/golden/
paper_curves.json, each entry citing its section)."""

import json
import os

import numpy as np
import pytest

from oracle import curves

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_curves.json")))


def test_uniform_frequency_curve():
    c = GOLD["frequency_curve_uniform"]
    f = curves.frequencies(c["n_steps"], c["stepsize"], c["s0"], c["nodes"])
    assert np.allclose(f, c["frequencies"], rtol=0, atol=1e-9)


def test_third_octave_curve():
    c = GOLD["frequency_curve_third_octave"]
    f = curves.frequencies(c["n_steps"], c["stepsize"], c["s0"], c["nodes"])
    assert len(f) == 24
    # every third step lands on a band centre (a node)
    for n in range(3, 25, 3):
        assert f[n - 1] == pytest.approx(c["nodes"][n // 3][1], abs=1e-12)
    # the steps between are on the straight line between the two centres
    for n in range(1, 25):
        lo, hi = c["nodes"][(n - 1) // 3], c["nodes"][(n - 1) // 3 + 1]
        t = (n - lo[0]) / (hi[0] - lo[0])
        assert f[n - 1] == pytest.approx(lo[1] + t * (hi[1] - lo[1]), abs=1e-12)
    # frequencies increase along the curve
    assert all(b > a for a, b in zip(f, f[1:]))


def _piece(pieces, s):
    for s_lo, s_hi, a, s_ref, slope in pieces:
        if s_lo <= s <= s_hi:
            return a + slope * (s - s_ref)
    raise AssertionError(s)


def test_admittance_curves_match_printed_pieces():
    c = GOLD["admittance_curves"]
    v0 = complex(0.3, -0.7)
    for s in np.linspace(0.0, 8.0, 33):
        c1 = _piece(c["c1_pieces"], s)
        c2 = _piece(c["c2_pieces"], s)
        a = curves.admittance(s, v0, c["curve1"], c["curve2"])
        assert a.real == pytest.approx(c1 * v0.real, abs=1e-14)
        assert a.imag == pytest.approx(c2 * v0.imag, abs=1e-14)
    # beyond curve 1's last node only curve 2 is defined
    with pytest.raises(ValueError):
        curves.admittance(9.0, v0, c["curve1"], c["curve2"])
    assert curves.admittance(9.0, v0, None, c["curve2"]).real == v0.real


def test_no_curve_is_factor_one_and_bad_nodes_fail():
    assert curves.admittance(4.2, 1.5 - 2j) == 1.5 - 2j
    with pytest.raises(ValueError):
        curves.curve_value([[0.0, 1.0], [0.0, 2.0]], 0.0)
    with pytest.raises(ValueError):
        curves.curve_value([[0.0, 1.0]], 0.0)
    with pytest.raises(ValueError):
        curves.curve_value([[0.0, 1.0], [1.0, 2.0]], -0.5)
