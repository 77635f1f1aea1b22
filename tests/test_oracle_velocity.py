"""Pin of the oracle's prescribed-velocity (VELO) right-hand side against the
pulsating sphere: uniform normal velocity u on a sphere of radius a radiates
p(a) = rho c u (i k a)/(i k a - 1) (time factor exp(-i w t); from the outgoing
monopole and Euler's equation).  The collocation solution converges to it at
first order in the element size: a wrong sign, a missing i k rho c factor or
a missing diagonal term of V would leave an O(1) error."""

import numpy as np

import synth
from oracle import velocity
from oracle.geometry import element_geometry
from oracle.presets import preset


def _err(level, k, rho_c=415.0, u0=1e-3):
    nodes, tris = synth.icosphere(level)
    g = element_geometry(nodes, tris)
    p = velocity.solve_velocity(g, k, np.full(len(tris), u0 + 0j), rho_c, p=preset("tight"))
    exact = rho_c * u0 * (1j * k) / (1j * k - 1.0)
    return np.max(np.abs(p - exact)) / abs(exact)


def test_pulsating_sphere_converges():
    e2, e3 = _err(2, 2.0), _err(3, 2.0)
    assert e3 < 0.03
    assert e3 < 0.65 * e2
