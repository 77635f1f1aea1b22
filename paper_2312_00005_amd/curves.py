"""Frequency steps and frequency-dependent admittances (host side).

The paper's input description (appendix) defines the frequencies of a run by
a piecewise-linear curve of the frequency step s, evaluated at
s_n = s0 + h n for n = 1 .. nSteps (Eq. (Freqcurve)), and lets an admittance
condition scale the real and imaginary part of its value v0 by two more such
curves of the same step: alpha(s) = c1(s) Re v0 + i c2(s) Im v0 (section on
frequency curves for admittance).  A missing curve means the factor 1.  A step
outside a curve's nodes is refused (the text does not extrapolate).

``AdmittanceGroup`` ties a set of elements to one such condition; the
frequency sweep turns the groups into the per-element admittance of each
step (the library takes beta = rho c Y per element).
"""

import bisect
from dataclasses import dataclass
from typing import Optional, Sequence, Tuple

import numpy as np

Node = Tuple[float, float]


class Curve:
    """Piecewise-linear curve through nodes (s_i, v_i) with increasing s_i."""

    def __init__(self, nodes: Sequence[Node]):
        pts = [(float(a), float(b)) for a, b in nodes]
        if len(pts) < 2:
            raise ValueError("a curve needs at least two nodes")
        if any(not s1 > s0 for (s0, _), (s1, _) in zip(pts, pts[1:])):
            raise ValueError("curve nodes must have increasing steps")
        self.s = [p[0] for p in pts]
        self.v = [p[1] for p in pts]

    def __call__(self, s: float) -> float:
        s = float(s)
        if s < self.s[0] or s > self.s[-1]:
            raise ValueError(f"step {s} lies outside the curve's nodes [{self.s[0]}, {self.s[-1]}]")
        # segment i spans [s[i], s[i+1]]; a step on an interior node takes the
        # segment to its left (both give the node's value)
        i = min(max(bisect.bisect_left(self.s, s) - 1, 0), len(self.s) - 2)
        t = (s - self.s[i]) / (self.s[i + 1] - self.s[i])
        return self.v[i] + t * (self.v[i + 1] - self.v[i])


def steps(n_steps: int, stepsize: float, s0: float) -> np.ndarray:
    """Frequency-step arguments s_n = s0 + stepsize n, n = 1 .. n_steps."""
    return s0 + stepsize * np.arange(1, n_steps + 1, dtype=np.float64)


def frequencies(n_steps: int, stepsize: float, s0: float, curve: Curve) -> np.ndarray:
    return np.array([curve(s) for s in steps(n_steps, stepsize, s0)])


@dataclass
class AdmittanceGroup:
    """Elements (indices into the mesh's triangles) with admittance v0, whose
    real and imaginary parts follow curve_re and curve_im (None: constant).
    The same scaling serves a source strength (elements unused)."""
    elements: np.ndarray
    v0: complex
    curve_re: Optional[Curve] = None
    curve_im: Optional[Curve] = None

    def value(self, s: float) -> complex:
        v0 = complex(self.v0)
        c1 = 1.0 if self.curve_re is None else self.curve_re(s)
        c2 = 1.0 if self.curve_im is None else self.curve_im(s)
        return complex(c1 * v0.real, c2 * v0.imag)


def element_admittance(groups: Sequence[AdmittanceGroup], n_elements: int, s: float) -> np.ndarray:
    """Admittance of every element at step s (0 where no group applies: sound
    hard); a later group overrides an earlier one on shared elements."""
    y = np.zeros(n_elements, dtype=np.complex128)
    for g in groups:
        idx = np.asarray(g.elements, dtype=np.int64)
        if idx.size and (idx.min() < 0 or idx.max() >= n_elements):
            raise ValueError("admittance group names an element outside the mesh")
        y[idx] = g.value(s)
    return y
