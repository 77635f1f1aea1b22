"""Dense Burton-Miller collocation operator (oracle; test infrastructure only).

Eq. (SystemI) with tau = 1 (exterior problem) and lambda = 1/2 at the
centroids (Sec. 2.3):

    (phi - gamma v)/2 - (H - gamma E) phi + (G - gamma H') v = phi_inc - gamma v_inc,

gamma = i/k (Sec. 2.5).  Boundary conditions enter per element as v_j = c_j
phi_j: sound-hard c = 0 (the default of the appendix "The Mesh"); admittance
c = -tau i k beta with beta = rho c Y (reading: v = -tau Y p along the
outward normal, the absorbing sign on an exterior surface; the duct's
plane-wave solution of Sec. 5.3 fixes it for the interior problem).
Hence

    A_ij = (1 - gamma c_i)/2 delta_ij - (H_ij - gamma E_ij) + (G_ij - gamma H'_ij) c_j.

The unknown may be read as pressure p = i w rho phi (Eq. (utopandv)); A is
unchanged by that scaling, so sources are given as pressure amplitudes.

Right-hand sides (Sec. 2.4): plane wave P0 exp(i k d.x); point source
P0 exp(i k R)/(4 pi R); b = p_inc - gamma dp_inc/dn at the centroids.

Solve: LAPACK LU (zgetrf / zgetrs through scipy), the paper's direct
reference solver (Sec. 3.2, Sec. 5.1.3).

Pinned by: tests/test_oracle_operator.py -- modal eigenvalues of the sphere
(A P_n(cos theta) ~ lambda_n P_n(cos theta) with O(h) error), the analytic
rigid and impedance sphere solutions, reciprocity of point sources.
"""

import numpy as np
import scipy.linalg

from .geometry import element_geometry
from .integrals import offdiag_integrals, self_integrals


def coupling(k, gamma=None, p=None):
    """gamma: given explicitly, else from the preset p (gamma_re +
    i gamma_im_k / k), else the paper's i/k."""
    if gamma is not None:
        return gamma
    if p is not None and "gamma_im_k" in p:
        return p.get("gamma_re", 0.0) + 1j * p["gamma_im_k"] / k
    return 1j / k


def bc_factor(k, beta, tau=1):
    """c_j with v_j = c_j phi_j: 0 for sound-hard, -tau i k beta_j for
    admittance.  The normal velocity is v = -tau Y p along the outward mesh
    normal: absorbing on an exterior surface (tau = 1) and, on an interior
    problem (tau = -1, normals pointing out of the fluid), the condition of
    the duct of Sec. 5.3 whose closed-form solution p = -rho c exp(ikx)
    carries v = +p/(rho c) at the admittance end."""
    if beta is None:
        return None
    return -tau * 1j * k * np.asarray(beta, dtype=np.complex128)


def rows(geom, row_idx, k, beta=None, p=None, gamma=None, cols=None, stats=None, tau=1):
    """Rows ``row_idx`` of the dense operator A (optionally only ``cols``).
    tau = -1: the interior problem of Eq. (SystemI), every integral term
    negated and the jump term (phi - gamma v)/2 kept."""
    gamma = coupling(k, gamma, p)
    N = geom["x"].shape[0]
    c = np.zeros(N, dtype=np.complex128) if beta is None else bc_factor(k, beta, tau)
    row_idx = np.asarray(row_idx, dtype=np.int64)
    cols = np.arange(N) if cols is None else np.asarray(cols, dtype=np.int64)
    out = np.zeros((row_idx.size, cols.size), dtype=np.complex128)
    ii, jj = np.meshgrid(np.arange(row_idx.size), np.arange(cols.size), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    gi, gj = row_idx[ii], cols[jj]
    off = gi != gj
    ii, jj, gi, gj = ii[off], jj[off], gi[off], gj[off]
    block = 200000
    for s in range(0, gi.size, block):
        e = slice(s, s + block)
        I = offdiag_integrals(geom["x"][gi[e]], geom["n"][gi[e]], geom["P0"][gj[e]],
                              geom["P1"][gj[e]], geom["P2"][gj[e]], geom["n"][gj[e]],
                              geom["A"][gj[e]], k, p, stats=stats)
        IG, IH, IHp, IE = I
        out[ii[e], jj[e]] = tau * (-(IH - gamma * IE) + (IG - gamma * IHp) * c[gj[e]])
    # diagonal entries present in this block
    pos = {int(j): t for t, j in enumerate(cols)}
    diag_rows = [(r, pos[int(g)]) for r, g in enumerate(row_idx) if int(g) in pos]
    if diag_rows:
        sel = np.array([row_idx[r] for r, _ in diag_rows])
        sub = {key: geom[key][sel] for key in ("P0", "P1", "P2", "x", "n", "A")}
        Gs, Es = self_integrals(sub, k, p)
        for t, (r, cpos) in enumerate(diag_rows):
            ci = c[sel[t]]
            out[r, cpos] = 0.5 * (1.0 - gamma * ci) + tau * (gamma * Es[t] + Gs[t] * ci)
    return out


def dense(geom, k, beta=None, p=None, gamma=None, stats=None, tau=1):
    N = geom["x"].shape[0]
    return rows(geom, np.arange(N), k, beta, p, gamma, stats=stats, tau=tau)


def diagonal(geom, k, beta=None, p=None, gamma=None):
    """Diagonal entries A_ii (self terms plus the 1/2 jump term)."""
    gamma = coupling(k, gamma, p)
    N = geom["x"].shape[0]
    c = np.zeros(N, dtype=np.complex128) if beta is None else bc_factor(k, beta)
    Gs, Es = self_integrals(geom, k, p)
    return 0.5 * (1.0 - gamma * c) + gamma * Es + Gs * c


def rhs_plane_wave(geom, k, d, P0=1.0, gamma=None, p=None):
    gamma = coupling(k, gamma, p)
    d = np.asarray(d, dtype=np.float64)
    x, n = geom["x"], geom["n"]
    pinc = P0 * np.exp(1j * k * (x @ d))
    dn = 1j * k * (n @ d) * pinc
    return pinc - gamma * dn


def rhs_point_source(geom, k, xs, P0=1.0, gamma=None, p=None):
    gamma = coupling(k, gamma, p)
    xs = np.asarray(xs, dtype=np.float64)
    x, n = geom["x"], geom["n"]
    Rv = x - xs
    R = np.linalg.norm(Rv, axis=1)
    pinc = P0 * np.exp(1j * k * R) / (4.0 * np.pi * R)
    dn = pinc * (1j * k - 1.0 / R) * np.sum(Rv * n, axis=1) / R
    return pinc - gamma * dn


def lu_solve(A, b):
    lu = scipy.linalg.lu_factor(A)
    return scipy.linalg.lu_solve(lu, b)


def solve(nodes, tris, k, beta=None, p=None, rhs=None, gamma=None):
    """Assemble, factor and solve; returns (p, geom, A)."""
    geom = element_geometry(nodes, tris)
    A = dense(geom, k, beta, p, gamma)
    return lu_solve(A, rhs), geom, A


def velocity(pressure, beta, rho_c, tau=1):
    """Normal particle velocity v = -tau Y p (Y = beta/(rho c)) along the
    outward normal; zero on sound-hard elements."""
    if beta is None:
        return np.zeros_like(pressure)
    return -tau * np.asarray(beta) / rho_c * pressure
