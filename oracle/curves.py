"""Frequency-step curves of the input description (oracle's own copy; test
infrastructure only: nothing in the library imports this module).

Appendix, input file:
* Frequency-defining curves (Sec. "Frequency-defining curves", Eq.
  (Freqcurve)): a piecewise-linear map from the frequency step s to the
  frequency; step n = 1 .. nSteps is evaluated at s_n = s0 + h n, with h the
  step size and s0 the start index.
* Admittance curves (Sec. "Frequency definition curves for admittance"): two
  piecewise-linear curves c1, c2 of the same step s scale the real and the
  imaginary part of an ADMI value v0: alpha(s) = c1(s) Re v0 + i c2(s) Im v0.
  A curve identifier of -1 means no frequency dependence (factor 1).

Readings (the text is silent on them): a step outside the nodes of a curve is
an error rather than an extrapolation; nodes must have strictly increasing
steps.  Each function is written as a plain scan over the segments so that it
can be checked against the paper by eye.
"""


def curve_value(nodes, s):
    """Value of the piecewise-linear curve through nodes [(s_0, v_0), ...] at s."""
    if len(nodes) < 2:
        raise ValueError("a curve needs at least two nodes")
    for (a, _), (b, _) in zip(nodes[:-1], nodes[1:]):
        if not b > a:
            raise ValueError("curve nodes must have increasing steps")
    for (s_lo, v_lo), (s_hi, v_hi) in zip(nodes[:-1], nodes[1:]):
        if s_lo <= s <= s_hi:
            # the line through the two bracketing nodes
            return v_lo + (v_hi - v_lo) / (s_hi - s_lo) * (s - s_lo)
    raise ValueError(f"step {s} lies outside the curve's nodes [{nodes[0][0]}, {nodes[-1][0]}]")


def step_arguments(n_steps, stepsize, s0):
    """s_n = s0 + stepsize * n for n = 1 .. n_steps (Eq. (Freqcurve))."""
    return [s0 + stepsize * n for n in range(1, n_steps + 1)]


def frequencies(n_steps, stepsize, s0, nodes):
    """f_n of every frequency step from the frequency-defining curve."""
    return [curve_value(nodes, s) for s in step_arguments(n_steps, stepsize, s0)]


def admittance(s, v0, nodes_re=None, nodes_im=None):
    """alpha(s) = c1(s) Re v0 + i c2(s) Im v0; a missing curve is the factor 1."""
    v0 = complex(v0)
    c1 = 1.0 if nodes_re is None else curve_value(nodes_re, s)
    c2 = 1.0 if nodes_im is None else curve_value(nodes_im, s)
    return complex(c1 * v0.real, c2 * v0.imag)
