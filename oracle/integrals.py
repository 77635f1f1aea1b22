"""Element integrals of G, H, H', E (oracle; test infrastructure only).

Follows Sec. 3.1 "Quadrature":

* i == j, singular (Sec. 3.1.1): G_ii by the six-triangle Duffy rule with an
  n x n Gauss-Legendre product on each sub-triangle; H_ii = H'_ii = 0 because
  y - x lies in the element's plane.
* i == j, hypersingular (Sec. 3.1.2): E_ii as the sum over the element's
  edges (traversed counter-clockwise about n) of the line integral of
  (n x grad_y G) . dy, plus k^2 G_ii.  Each edge is cut into equal parts
  with a Gauss-Legendre rule on each.
* i != j (Sec. 3.1.3-3.1.4): with r~ = |x_i - mid(T)| / sqrt(A_T) for the
  (sub-)element T (mid = vertex mean), T is split into four children
  through its edge midpoints while r~ < ``subdiv_ratio``; more than
  ``max_subdiv`` nested splits is an error.  Otherwise the order m is the
  smallest m >= 1 for which the three a-priori estimates
      32 q^(2m+1),  64 (2m+1) q^(2m+2),  128 (m+1)(2m+1) q^(2m+3),  q = 1/(2 r~)
  are all below ``quad_eps``; if m exceeds ``m_max`` it is capped (paper
  default) or T is split once more (``split_on_cap``, the higher-accuracy
  variant of Sec. 5.1.2).  The conical rule of order m is then applied.

Children of T = (P0, P1, P2) with edge midpoints M01, M12, M20:
  (P0, M01, M20), (P1, M12, M01), (P2, M20, M12), (M01, M12, M20).

Pinned by: tests/test_oracle_integrals.py -- static closed forms (k = 0) for
the self terms, the off-plane limit for E_ii, adaptive brute-force
quadrature (scipy) for regular and subdivided pairs, exact zeros for
H_ii and H'_ii.
"""

import numpy as np

from .kernels import FOUR_PI, kernels
from .rules import conical, gauss_legendre01, edge_rule


class SubdivisionError(RuntimeError):
    def __init__(self, pair_index):
        super().__init__(f"more than the allowed number of nested subdivisions "
                         f"for pair index {pair_index}")
        self.pair_index = int(pair_index)


def estimator_order(rt, eps, m_limit=64):
    """Smallest m >= 1 with all three a-priori error estimates below eps
    (Sec. 3.1.4).  ``rt`` is r~ (array)."""
    rt = np.asarray(rt, dtype=np.float64)
    q = 1.0 / (2.0 * rt)
    m_out = np.full(rt.shape, m_limit, dtype=np.int64)
    done = np.zeros(rt.shape, dtype=bool)
    for m in range(1, m_limit + 1):
        eg = 32.0 * q ** (2 * m + 1)
        eh = 64.0 * (2 * m + 1) * q ** (2 * m + 2)
        ee = 128.0 * (m + 1) * (2 * m + 1) * q ** (2 * m + 3)
        ok = (eg < eps) & (eh < eps) & (ee < eps) & ~done
        m_out[ok] = m
        done |= ok
        if done.all():
            break
    return m_out


def _apply_rule(x, nx, v0, v1, v2, ny, area, m, k, chunk=20000):
    """Conical rule of order m on the triangles (v0, v1, v2); returns the
    four integrals (n_items,) each."""
    a, b, w = conical(m)
    n = x.shape[0]
    out = np.empty((4, n), dtype=np.complex128)
    for s in range(0, n, chunk):
        e = slice(s, min(n, s + chunk))
        y = (v0[e, None, :] + a[None, :, None] * (v1[e] - v0[e])[:, None, :]
             + b[None, :, None] * (v2[e] - v0[e])[:, None, :])
        G, H, Hp, E = kernels(x[e, None, :], nx[e, None, :], y, ny[e, None, :], k)
        ww = (2.0 * area[e])[:, None] * w[None, :]
        out[0, e] = np.sum(G * ww, axis=1)
        out[1, e] = np.sum(H * ww, axis=1)
        out[2, e] = np.sum(Hp * ww, axis=1)
        out[3, e] = np.sum(E * ww, axis=1)
    return out


def offdiag_integrals(x, nx, P0, P1, P2, ny, A, k, p, stats=None):
    """Integrals over elements that do not contain the collocation node.

    All inputs are per pair: x, nx (P,3) collocation node and its normal;
    P0, P1, P2 (P,3) the source triangle; ny (P,3) its normal; A (P,) its
    area.  Returns a (4, P) complex array (I^G, I^H, I^H', I^E)."""
    P = x.shape[0]
    out = np.zeros((4, P), dtype=np.complex128)
    idx = np.arange(P)
    v0, v1, v2 = P0.copy(), P1.copy(), P2.copy()
    area = np.asarray(A, dtype=np.float64).copy()
    depth = np.zeros(P, dtype=np.int64)
    n_points = 0
    n_items = 0
    while idx.size:
        mid = (v0 + v1 + v2) / 3.0
        d = x[idx] - mid
        rt = np.sqrt(np.sum(d * d, axis=1)) / np.sqrt(area)
        split = rt < p["subdiv_ratio"]
        m = np.ones(idx.size, dtype=np.int64)
        reg = ~split
        if reg.any():
            m[reg] = estimator_order(rt[reg], p["quad_eps"])
        over = reg & (m > p["m_max"])
        if p["split_on_cap"]:
            split |= over
        else:
            m[over] = p["m_max"]
        if np.any(split & (depth >= p["max_subdiv"])):
            bad = idx[np.nonzero(split & (depth >= p["max_subdiv"]))[0][0]]
            raise SubdivisionError(bad)
        ready = ~split
        for mv in np.unique(m[ready]):
            sel = np.nonzero(ready & (m == mv))[0]
            ii = idx[sel]
            vals = _apply_rule(x[ii], nx[ii], v0[sel], v1[sel], v2[sel],
                               ny[ii], area[sel], int(mv), k)
            n_points += sel.size * int(mv) * int(mv)
            n_items += sel.size
            for q in range(4):
                np.add.at(out[q], ii, vals[q])
        s = np.nonzero(split)[0]
        if s.size == 0:
            break
        a0, a1, a2 = v0[s], v1[s], v2[s]
        m01, m12, m20 = 0.5 * (a0 + a1), 0.5 * (a1 + a2), 0.5 * (a2 + a0)
        v0 = np.concatenate([a0, a1, a2, m01])
        v1 = np.concatenate([m01, m12, m20, m12])
        v2 = np.concatenate([m20, m01, m12, m20])
        idx = np.tile(idx[s], 4)
        area = np.tile(area[s] * 0.25, 4)
        depth = np.tile(depth[s] + 1, 4)
    if stats is not None:
        stats["points"] = stats.get("points", 0) + n_points
        stats["items"] = stats.get("items", 0) + n_items
    return out


def self_integrals(geom, k, p):
    """(G_ii, E_ii) for every element (H_ii = H'_ii = 0 exactly)."""
    P0, P1, P2, x, n = geom["P0"], geom["P1"], geom["P2"], geom["x"], geom["n"]
    N = x.shape[0]
    u, wu = gauss_legendre01(p["self_n"])
    U, V = np.meshgrid(u, u, indexing="ij")
    W = np.outer(wu, wu)
    U, V, W = U.ravel(), V.ravel(), W.ravel()
    M01, M12, M20 = 0.5 * (P0 + P1), 0.5 * (P1 + P2), 0.5 * (P2 + P0)
    subs = [(P0, M01), (M01, P1), (P1, M12), (M12, P2), (P2, M20), (M20, P0)]
    Gs = np.zeros(N, dtype=np.complex128)
    for Q1, Q2 in subs:
        As = 0.5 * np.linalg.norm(np.cross(Q1 - x, Q2 - x), axis=1)
        y = x[:, None, :] + U[None, :, None] * ((Q1 - x)[:, None, :]
                                                + V[None, :, None] * (Q2 - Q1)[:, None, :])
        R = y - x[:, None, :]
        r = np.sqrt(np.sum(R * R, axis=2))
        G = np.exp(1j * k * r) / (FOUR_PI * r)
        Gs += np.sum(G * (2.0 * As)[:, None] * (U * W)[None, :], axis=1)
    t, wt = edge_rule(p["edge_parts"], p["edge_gauss"])
    Es = np.zeros(N, dtype=np.complex128)
    for Pa, Pb in ((P0, P1), (P1, P2), (P2, P0)):
        dvec = Pb - Pa
        y = Pa[:, None, :] + t[None, :, None] * dvec[:, None, :]
        R = y - x[:, None, :]
        r = np.sqrt(np.sum(R * R, axis=2))
        G = np.exp(1j * k * r) / (FOUR_PI * r)
        grad = (G * (1j * k - 1.0 / r) / r)[:, :, None] * R
        integrand = np.sum(np.cross(n[:, None, :], grad) * dvec[:, None, :], axis=2)
        Es += np.sum(integrand * wt[None, :], axis=1)
    Es += k * k * Gs
    return Gs, Es
