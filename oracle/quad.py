"""Plane quadrilateral elements and meshes of triangles and quadrilaterals
(oracle; test infrastructure only).

Sec. 2.2: the elements are flat triangles or plane quadrilaterals with one
constant value each.  Sec. 2.3: the collocation node is the mean of the
element's vertex coordinates.  A mesh is an (N, 4) vertex index array whose
fourth entry is negative on triangles; vertices run counter-clockwise about
the outward normal (appendix "The Mesh").  For a plane quadrilateral
P0 P1 P2 P3 the normal is the unit vector along (P2 - P0) x (P3 - P1) and the
area half the length of that cross product.

Integrals over a quadrilateral (Sec. 3.1):

* singular (Sec. 3.1.1): eight sub-triangles sharing the collocation node
  (the node joined to the four vertices and the four edge midpoints), each
  with the Duffy map y = x + u [(Q1 - x) + v (Q2 - Q1)] and n x n
  Gauss-Legendre in u, v; H_ii = H'_ii = 0 (y - x lies in the plane);
* hypersingular (Sec. 3.1.2): the line integrals over the four edges plus
  k^2 G_ii, as for triangles;
* regular and nearly singular (Sec. 3.1.3-3.1.4): r~ = |x - mid| / sqrt(A)
  with mid the vertex mean; the element is split into four through its edge
  midpoints and its vertex mean while r~ < ``subdiv_ratio``; otherwise the
  order m follows from the same three estimates as for triangles and the
  m x m Gauss-Legendre product on [-1, 1]^2 is applied through the bilinear
  map y = sum_a N_a(xi, eta) P_a (Abramowitz-Stegun Table 25.4 nodes), with
  the Jacobian |dy/dxi x dy/deta|.

Triangles of a mixed mesh use oracle.integrals unchanged.

Pinned by: tests/test_oracle_quad.py -- exactness of the product rule on
parallelograms and trapezoids, self terms against the polar closed forms,
off-diagonal integrals of a quadrilateral against the sum over its two
triangles (computed by the triangle rules), the rigid sphere of plane
quadrilaterals and pole triangles against the analytic series, and the duct
of Sec. 5.3 meshed with rectangles against its plane-wave solution.
"""

import numpy as np

from .integrals import SubdivisionError, estimator_order, offdiag_integrals, self_integrals
from .kernels import FOUR_PI, kernels
from .operator import bc_factor, coupling
from .rules import edge_rule, gauss_legendre01


def mixed_geometry(nodes, elems):
    """Per element: vertices V (N, 4, 3) (V[:, 3] = V[:, 2] on triangles),
    is_quad (N,), collocation node x, unit normal n, area A, and P0, P1, P2
    (the first three vertices)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    elems = np.asarray(elems, dtype=np.int64)
    is_quad = elems[:, 3] >= 0
    i3 = np.where(is_quad, elems[:, 3], elems[:, 2])
    V = np.stack([nodes[elems[:, 0]], nodes[elems[:, 1]], nodes[elems[:, 2]], nodes[i3]], axis=1)
    P0, P1, P2, P3 = V[:, 0], V[:, 1], V[:, 2], V[:, 3]
    cr_t = np.cross(P1 - P0, P2 - P0)
    cr_q = np.cross(P2 - P0, P3 - P1)
    cr = np.where(is_quad[:, None], cr_q, cr_t)
    nrm = np.linalg.norm(cr, axis=1)
    x = np.where(is_quad[:, None], 0.25 * (P0 + P1 + P2 + P3), (P0 + P1 + P2) / 3.0)
    return {"V": V, "is_quad": is_quad, "x": x, "n": cr / nrm[:, None], "A": 0.5 * nrm,
            "P0": P0, "P1": P1, "P2": P2}


def product_rule(m):
    """m x m Gauss-Legendre on [-1, 1]^2: (xi, eta, w), length m*m."""
    g, w = np.polynomial.legendre.leggauss(m)
    XI, ETA = np.meshgrid(g, g, indexing="ij")
    return XI.ravel(), ETA.ravel(), np.outer(w, w).ravel()


def bilinear(V, xi, eta):
    """Points y (..., npts, 3) and Jacobians |y_xi x y_eta| (..., npts) of the
    bilinear map of quadrilaterals V (..., 4, 3) at (xi, eta)."""
    N = np.stack([(1 - xi) * (1 - eta), (1 + xi) * (1 - eta), (1 + xi) * (1 + eta), (1 - xi) * (1 + eta)], 0) / 4
    dxi = np.stack([-(1 - eta), (1 - eta), (1 + eta), -(1 + eta)], 0) / 4
    deta = np.stack([-(1 - xi), -(1 + xi), (1 + xi), (1 - xi)], 0) / 4
    y = np.einsum("aq,...ad->...qd", N, V)
    yx = np.einsum("aq,...ad->...qd", dxi, V)
    ye = np.einsum("aq,...ad->...qd", deta, V)
    J = np.linalg.norm(np.cross(yx, ye), axis=-1)
    return y, J


def _apply_product(x, nx, V, ny, m, k, chunk=20000):
    xi, eta, w = product_rule(m)
    n = x.shape[0]
    out = np.empty((4, n), dtype=np.complex128)
    for s in range(0, n, chunk):
        e = slice(s, min(n, s + chunk))
        y, J = bilinear(V[e], xi, eta)
        G, H, Hp, E = kernels(x[e, None, :], nx[e, None, :], y, ny[e, None, :], k)
        ww = J * w[None, :]
        out[0, e] = np.sum(G * ww, axis=1)
        out[1, e] = np.sum(H * ww, axis=1)
        out[2, e] = np.sum(Hp * ww, axis=1)
        out[3, e] = np.sum(E * ww, axis=1)
    return out


def quad_area(V):
    return 0.5 * np.linalg.norm(np.cross(V[..., 2, :] - V[..., 0, :], V[..., 3, :] - V[..., 1, :]), axis=-1)


def offdiag_quad(x, nx, V, ny, k, p):
    """Integrals (I^G, I^H, I^H', I^E), shape (4, P), over the quadrilaterals
    V (P, 4, 3) (normals ny) from collocation nodes x (normals nx) that do not
    lie in them."""
    P = x.shape[0]
    out = np.zeros((4, P), dtype=np.complex128)
    idx = np.arange(P)
    Q = np.array(V, dtype=np.float64)
    area = quad_area(Q)
    depth = np.zeros(P, dtype=np.int64)
    while idx.size:
        mid = Q.mean(axis=1)
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
            raise SubdivisionError(idx[np.nonzero(split & (depth >= p["max_subdiv"]))[0][0]])
        ready = ~split
        for mv in np.unique(m[ready]):
            sel = np.nonzero(ready & (m == mv))[0]
            ii = idx[sel]
            vals = _apply_product(x[ii], nx[ii], Q[sel], ny[ii], int(mv), k)
            for q in range(4):
                np.add.at(out[q], ii, vals[q])
        s = np.nonzero(split)[0]
        if s.size == 0:
            break
        A0, A1, A2, A3 = Q[s, 0], Q[s, 1], Q[s, 2], Q[s, 3]
        M01, M12, M23, M30 = 0.5 * (A0 + A1), 0.5 * (A1 + A2), 0.5 * (A2 + A3), 0.5 * (A3 + A0)
        C = 0.25 * (A0 + A1 + A2 + A3)
        Q = np.concatenate([np.stack(c, axis=1) for c in
                            ((A0, M01, C, M30), (M01, A1, M12, C), (C, M12, A2, M23), (M30, C, M23, A3))])
        idx = np.tile(idx[s], 4)
        area = quad_area(Q)
        depth = np.tile(depth[s] + 1, 4)
    return out


def self_quad(V, x, n, k, p):
    """(G_ii, E_ii) of quadrilaterals V (N, 4, 3) with collocation nodes x
    and normals n."""
    N = x.shape[0]
    u, wu = gauss_legendre01(p["self_n"])
    U, W = np.meshgrid(u, u, indexing="ij")
    Wt = np.outer(wu, wu).ravel()
    U, Vv = U.ravel(), W.ravel()
    corners = [V[:, a] for a in range(4)]
    mids = [0.5 * (V[:, a] + V[:, (a + 1) % 4]) for a in range(4)]
    subs = []
    for a in range(4):
        subs += [(corners[a], mids[a]), (mids[a], corners[(a + 1) % 4])]
    Gs = np.zeros(N, dtype=np.complex128)
    for Q1, Q2 in subs:
        As = 0.5 * np.linalg.norm(np.cross(Q1 - x, Q2 - x), axis=1)
        y = x[:, None, :] + U[None, :, None] * ((Q1 - x)[:, None, :] + Vv[None, :, None] * (Q2 - Q1)[:, None, :])
        r = np.linalg.norm(y - x[:, None, :], axis=2)
        G = np.exp(1j * k * r) / (FOUR_PI * r)
        Gs += np.sum(G * (2.0 * As)[:, None] * (U * Wt)[None, :], axis=1)
    t, wt = edge_rule(p["edge_parts"], p["edge_gauss"])
    Es = np.zeros(N, dtype=np.complex128)
    for a in range(4):
        Pa, Pb = corners[a], corners[(a + 1) % 4]
        dvec = Pb - Pa
        y = Pa[:, None, :] + t[None, :, None] * dvec[:, None, :]
        R = y - x[:, None, :]
        r = np.sqrt(np.sum(R * R, axis=2))
        G = np.exp(1j * k * r) / (FOUR_PI * r)
        grad = (G * (1j * k - 1.0 / r) / r)[:, :, None] * R
        Es += np.sum(np.sum(np.cross(n[:, None, :], grad) * dvec[:, None, :], axis=2) * wt[None, :], axis=1)
    return Gs, Es + k * k * Gs


def element_integrals(geom, xs, nxs, cols, k, p):
    """(4, P) integrals over elements cols (P,) from points xs (P, 3) with
    normals nxs (P, 3); no point may lie in its element."""
    cols = np.asarray(cols, dtype=np.int64)
    out = np.zeros((4, cols.size), dtype=np.complex128)
    q = geom["is_quad"][cols]
    t = ~q
    if t.any():
        j = cols[t]
        out[:, t] = offdiag_integrals(xs[t], nxs[t], geom["P0"][j], geom["P1"][j], geom["P2"][j],
                                      geom["n"][j], geom["A"][j], k, p)
    if q.any():
        j = cols[q]
        out[:, q] = offdiag_quad(xs[q], nxs[q], geom["V"][j], geom["n"][j], k, p)
    return out


def self_terms(geom, sel, k, p):
    """(G_ii, E_ii) of elements sel."""
    sel = np.asarray(sel, dtype=np.int64)
    Gs = np.zeros(sel.size, dtype=np.complex128)
    Es = np.zeros(sel.size, dtype=np.complex128)
    q = geom["is_quad"][sel]
    if (~q).any():
        j = sel[~q]
        sub = {key: geom[key][j] for key in ("P0", "P1", "P2", "x", "n", "A")}
        Gs[~q], Es[~q] = self_integrals(sub, k, p)
    if q.any():
        j = sel[q]
        Gs[q], Es[q] = self_quad(geom["V"][j], geom["x"][j], geom["n"][j], k, p)
    return Gs, Es


def rows(geom, row_idx, k, beta=None, p=None, gamma=None, tau=1):
    """Rows of the Burton-Miller operator of Eq. (SystemI) on a mixed mesh
    (the same entries as oracle.operator.rows, element integrals by type)."""
    gamma = coupling(k, gamma, p)
    N = geom["x"].shape[0]
    c = np.zeros(N, dtype=np.complex128) if beta is None else bc_factor(k, beta, tau)
    row_idx = np.asarray(row_idx, dtype=np.int64)
    out = np.zeros((row_idx.size, N), dtype=np.complex128)
    ii, jj = np.meshgrid(np.arange(row_idx.size), np.arange(N), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    gi = row_idx[ii]
    off = gi != jj
    ii, jj, gi = ii[off], jj[off], gi[off]
    block = 200000
    for s in range(0, gi.size, block):
        e = slice(s, s + block)
        IG, IH, IHp, IE = element_integrals(geom, geom["x"][gi[e]], geom["n"][gi[e]], jj[e], k, p)
        out[ii[e], jj[e]] = tau * (-(IH - gamma * IE) + (IG - gamma * IHp) * c[jj[e]])
    Gs, Es = self_terms(geom, row_idx, k, p)
    ci = c[row_idx]
    out[np.arange(row_idx.size), row_idx] = 0.5 * (1.0 - gamma * ci) + tau * (gamma * Es + Gs * ci)
    return out


def dense(geom, k, beta=None, p=None, gamma=None, tau=1):
    return rows(geom, np.arange(geom["x"].shape[0]), k, beta, p, gamma, tau)


def field_pv(geom, pts, k, p_surf, dpdn_surf, p=None, tau=1):
    """Pressure at field points off the surface by the representation formula
    (Eq. (BIE_I) with lambda = 1), without the incident field:
    tau sum_j (I^H_j(x) p_j - I^G_j(x) v_j)."""
    pts = np.asarray(pts, dtype=np.float64)
    N = geom["x"].shape[0]
    out = np.zeros(pts.shape[0], dtype=np.complex128)
    zero_n = np.zeros((N, 3))
    for i, xp in enumerate(pts):
        I = element_integrals(geom, np.broadcast_to(xp, (N, 3)).copy(), zero_n, np.arange(N), k, p)
        out[i] = tau * (np.sum(I[1] * p_surf) - np.sum(I[0] * dpdn_surf))
    return out
