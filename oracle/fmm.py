"""Cluster tree and multilevel FMM in plain steps (oracle; test infrastructure only).

Cluster tree (Sec. 3.3.2 "Cluster generation", Sec. 3.3.4 "Multi level FMM"):
  * a group of elements is split by a box around its vertices, every axis cut
    into max(1, floor(extent/edge + 1/2)) equal slabs; an element goes to the
    sub-box holding its centroid; empty boxes are dropped; boxes are ordered
    lexicographically (x, y, z);
  * midpoint = mean over the vertex incidences of the cluster's elements,
    radius = largest vertex distance from the midpoint (footnote to Eq.
    (FMMTruncation));
  * small clusters (radius below half the group's mean radius, or fewer than
    leaf_size/4 elements) are merged into the nearest non-small cluster of
    the group ("merged with the nearest cluster with large size");
  * level 1 splits the mesh with edge e_r, level l splits each level-(l-1)
    cluster with edge e_r / 2^(l-1); all leaves are on the last level; the
    default leaf edge is sqrt(leaf_size * mean element area);
  * far pairs: |z_i - z_j| > a (r_i + r_j) (Eq. (Farfieldcond), a = 2/sqrt(3)
    in the paper); level 1 interacts with all far clusters; on level l > 1 the
    candidates are the children of the parent's near clusters (the
    interaction list), near pairs remain only on the leaf level.

Expansion (Eq. (FMMBase), Sec. 3.3.1), read with sphere weights summing to
4 pi and prefactor i k / (16 pi^2):
  G(x, y) ~ ik/(16 pi^2) sum_nu w_nu exp(ik (x - z_m).s) D_L(z_m - z_n, s)
                                       exp(ik (z_n - y).s)
  D_L(X, s) = sum_{l=0}^{L} i^l (2l+1) h_l(k|X|) P_l(Xh . s),
with L Gauss-Legendre nodes in cos(theta) and 2L equally spaced azimuths.
Derivatives in y multiply by -ik s.n_y, in x by ik s.n_x, so for element j in
cluster n and node i in cluster m the far entry of A is
  ik/(16 pi^2) sum_nu w_nu (1 - gamma ik s.n_i) exp(ik (x_i - z_m).s) D_L
               * int_Gj exp(ik (z_n - y).s) dy (c_j + ik s.n_j).
The element integral uses the conical rule of order t_order.

Truncation length per level (Eq. (FMMTruncation)):
  l_mode 0 (paper): L = max(l_min, ceil(kd + l_factor log10(kd + pi))), kd = 2 r_max k;
  l_mode 1: additionally L >= ceil(kd + 1.8 digits^(2/3) (kd)^(1/3)) and
            L >= ceil(ln(eps) / ln(1/a)), digits = -log10(eps); then L is
            lowered (not below 4) while 2^-52 (2L+1) |h_L(k X_min)| > eps/10,
            X_min the smallest centre distance of the level's interaction
            pairs -- the small-argument growth of h_L (Sec. 4.2) would
            otherwise amplify rounding beyond the target.
  The complex-FP32 operator of the mixed path has its own lengths: the same
  rule with eps = fmm_eps_mixed and the cap taken with 2^-23 in every mode.

Between levels the signatures move by band-limited interpolation (the
alternative to stored per-level matrices named in Sec. 3.3.4 and planned in
the conclusions): values on a child grid are projected onto spherical
harmonics of degree < L_child with the child's quadrature and evaluated on
the parent grid, then shifted by exp(ik (z_parent - z_child).s).  The
downward pass applies the weighted transpose (anterpolation).  When parent and
child grids coincide the signatures are shifted without any resampling.

Pinned by: tests/test_oracle_fmm.py -- sphere quadrature integrates
spherical harmonics exactly, the expansion reproduces G for separated
points, interpolation is exact for band-limited functions, the tree
partitions all element pairs exactly once, and the FMM matvec agrees with
the dense operator to the expansion accuracy.
"""

import math

import numpy as np
from scipy.special import spherical_jn, spherical_yn, sph_harm_y

from .rules import conical
from .operator import coupling, bc_factor


# ------------------------------------------------------------------ tree ---

def _group_stats(geom, elems):
    v = np.stack([geom["P0"][elems], geom["P1"][elems], geom["P2"][elems]], axis=1).reshape(-1, 3)
    z = np.cumsum(v, axis=0)[-1] / (3.0 * len(elems))
    d = v - z
    r2 = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
    return z, math.sqrt(float(r2.max()))


def _split(geom, elems, edge):
    v = np.stack([geom["P0"][elems], geom["P1"][elems], geom["P2"][elems]], axis=1).reshape(-1, 3)
    lo = v.min(axis=0)
    hi = v.max(axis=0)
    ext = hi - lo
    n = np.maximum(1, np.floor(ext / edge + 0.5)).astype(np.int64)
    c = geom["x"][elems]
    idx = np.zeros((len(elems), 3), dtype=np.int64)
    for d in range(3):
        if n[d] == 1:
            continue
        t = (c[:, d] - lo[d]) * float(n[d]) / ext[d]
        idx[:, d] = np.clip(np.floor(t).astype(np.int64), 0, n[d] - 1)
    key = (idx[:, 0] * n[1] + idx[:, 1]) * n[2] + idx[:, 2]
    order = np.argsort(key, kind="stable")
    groups = []
    ks = key[order]
    start = 0
    for i in range(1, len(order) + 1):
        if i == len(order) or ks[i] != ks[start]:
            groups.append(np.asarray(elems)[order[start:i]])
            start = i
    return groups


def _merge(geom, groups, leaf_size):
    ng = len(groups)
    if ng <= 1:
        return groups
    stats = [_group_stats(geom, g) for g in groups]
    rsum = 0.0
    for _, r in stats:
        rsum += r
    rmean = rsum / ng
    nmin = max(1, leaf_size // 4)
    small = [(stats[i][1] < 0.5 * rmean) or (len(groups[i]) < nmin) for i in range(ng)]
    if not any(small) or all(small):
        return groups
    target = {}
    for i in range(ng):
        if not small[i]:
            continue
        best, bi = math.inf, -1
        for j in range(ng):
            if small[j]:
                continue
            d = stats[i][0] - stats[j][0]
            d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
            if d2 < best:
                best, bi = d2, j
        target[i] = bi
    out = []
    for j in range(ng):
        if small[j]:
            continue
        parts = [groups[j]] + [groups[i] for i in range(ng) if small[i] and target[i] == j]
        out.append(np.sort(np.concatenate(parts)))
    return out


class Tree:
    """levels[l] is a dict with keys groups, z, r, parent, children, near, il;
    perm concatenates the leaf groups (tree position -> element index)."""

    def __init__(self, levels, perm):
        self.levels = levels
        self.perm = perm


def build_tree(geom, levels, leaf_size, admissibility, root_edge=0.0):
    N = geom["x"].shape[0]
    if root_edge <= 0.0:
        asum = 0.0
        for a in geom["A"]:
            asum += float(a)
        leaf_edge = math.sqrt(float(leaf_size) * (asum / N))
        root_edge = leaf_edge * 2.0 ** (levels - 1)
    lv = []
    groups = _merge(geom, _split(geom, np.arange(N), root_edge), leaf_size)
    lv.append({"groups": groups, "parent": [-1] * len(groups)})
    for l in range(1, levels):
        edge = root_edge / 2.0 ** l
        gs, par = [], []
        for p, g in enumerate(lv[-1]["groups"]):
            ch = _merge(geom, _split(geom, g, edge), leaf_size)
            gs += ch
            par += [p] * len(ch)
        lv.append({"groups": gs, "parent": par})
    for L in lv:
        st = [_group_stats(geom, g) for g in L["groups"]]
        L["z"] = np.array([s[0] for s in st])
        L["r"] = np.array([s[1] for s in st])
    for l in range(levels - 1):
        ch = [[] for _ in lv[l]["groups"]]
        for c, p in enumerate(lv[l + 1]["parent"]):
            ch[p].append(c)
        lv[l]["children"] = ch
    lv[-1]["children"] = [[] for _ in lv[-1]["groups"]]

    def far(L, a, b):
        d = L["z"][a] - L["z"][b]
        d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
        lim = admissibility * (L["r"][a] + L["r"][b])
        return d2 > lim * lim

    for l, L in enumerate(lv):
        L["near"], L["il"] = [], []
        for c in range(len(L["groups"])):
            if l == 0:
                cand = range(len(L["groups"]))
            else:
                P = lv[l - 1]
                cand = [o for q in P["near"][L["parent"][c]] for o in P["children"][q]]
            nr, il = [], []
            for o in cand:
                (il if far(L, c, o) else nr).append(o)
            L["near"].append(nr)
            L["il"].append(il)
    perm = np.concatenate(lv[-1]["groups"])
    return Tree(lv, perm)


def default_levels(N):
    """Level count when none is given (Sec. 3.3.4): the printed formula is
    garbled; read as 1 + round(log2(sqrt(N) / 22.5) / 2), at least 1."""
    v = 0.5 * math.log2(math.sqrt(N) / 22.5)
    return max(1, 1 + math.floor(v + 0.5))


def pair_partition_counts(tree, N):
    """Count how often every (i, j) pair is covered by a leaf near pair or by
    an interaction-list pair on some level (each must be exactly once)."""
    cover = np.zeros((N, N), dtype=np.int32)
    for L in tree.levels:
        for c, g in enumerate(L["groups"]):
            for o in L["il"][c]:
                cover[np.ix_(g, L["groups"][o])] += 1
    leaf = tree.levels[-1]
    for c, g in enumerate(leaf["groups"]):
        for o in leaf["near"][c]:
            cover[np.ix_(g, leaf["groups"][o])] += 1
    return cover


# ------------------------------------------------------- expansion pieces ---

def hankel_abs(n, x):
    return math.hypot(float(spherical_jn(n, x)), float(spherical_yn(n, x)))


def truncation_length(k, r_max, p, x_min=None, single=False):
    """L of one level; x_min = smallest |z_m - z_n| over the level's
    interaction pairs (None: no pairs).  single=True gives the length of the
    complex-FP32 operator (accuracy fmm_eps_mixed, FP32 rounding)."""
    kd = 2.0 * r_max * k
    L = max(p["l_min"], math.ceil(kd + p["l_factor"] * math.log10(kd + math.pi)))
    eps = p["fmm_eps_mixed"] if single else p["fmm_eps"]
    unit = 2.0 ** -23 if single else 2.0 ** -52
    if p["l_mode"] == 1:
        digits = -math.log10(eps)
        L = max(L, math.ceil(kd + 1.8 * digits ** (2.0 / 3.0) * kd ** (1.0 / 3.0)))
        L = max(L, math.ceil(math.log(eps) / math.log(1.0 / p["admissibility"])))
    if x_min is not None and (p["l_mode"] == 1 or single):
        # stability: rounding amplified by (2L+1)|h_L(k X_min)| stays below eps/10
        x = k * x_min
        while L > 4 and unit * (2 * L + 1) * hankel_abs(L, x) > 0.1 * eps:
            L -= 1
    return L


def level_min_separation(level):
    best = None
    for m in range(len(level["groups"])):
        for n in level["il"][m]:
            d = level["z"][m] - level["z"][n]
            v = math.sqrt(float(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]))
            best = v if best is None else min(best, v)
    return best


def sphere_grid(L):
    """Nodes (2L*L, 3) and weights (sum 4 pi): L Gauss-Legendre nodes in
    cos(theta) times 2L azimuths phi_j = j pi / L; theta-major order."""
    x, w = np.polynomial.legendre.leggauss(L)
    phi = np.arange(2 * L) * math.pi / L
    ct = np.repeat(x, 2 * L)
    st = np.sqrt(1.0 - ct * ct)
    ph = np.tile(phi, L)
    s = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    return s, np.repeat(w, 2 * L) * (math.pi / L), x, phi


def hankel1(n, x):
    return spherical_jn(n, x) + 1j * spherical_yn(n, x)


def translation(k, X, s, L):
    """D_L(X, s) for one separation vector X and all nodes s (Eq. (FMMBase))."""
    Xn = np.linalg.norm(X)
    ct = s @ (X / Xn)
    out = np.zeros(s.shape[0], dtype=np.complex128)
    p_prev, p = np.ones_like(ct), ct
    for l in range(L + 1):
        Pl = np.ones_like(ct) if l == 0 else (ct if l == 1 else None)
        if l >= 2:
            p_next = ((2 * l - 1) * ct * p - (l - 1) * p_prev) / l
            p_prev, p = p, p_next
            Pl = p
        out += (1j ** l) * (2 * l + 1) * hankel1(l, k * Xn) * Pl
    return out


def translations(k, X, s, L):
    """D_L for many separation vectors X (P, 3) at all nodes s: (P, nu)."""
    Xn = np.linalg.norm(X, axis=1)
    ct = (X / Xn[:, None]) @ s.T
    out = np.zeros(ct.shape, dtype=np.complex128)
    p_prev = np.ones_like(ct)
    p = ct.copy()
    for l in range(L + 1):
        if l == 0:
            Pl = p_prev
        elif l == 1:
            Pl = p
        else:
            p_next = ((2 * l - 1) * ct * p - (l - 1) * p_prev) / l
            p_prev, p = p, p_next
            Pl = p
        out += ((1j ** l) * (2 * l + 1) * hankel1(l, k * Xn))[:, None] * Pl
    return out


def green_expansion(k, x, y, z1, z2, L):
    """The truncated, discretised expansion of G(x, y) about z1 (near x) and
    z2 (near y)."""
    s, w, _, _ = sphere_grid(L)
    D = translation(k, z1 - z2, s, L)
    return (1j * k / (16 * math.pi ** 2)) * np.sum(
        w * np.exp(1j * k * ((x - z1) @ s.T)) * D * np.exp(1j * k * ((z2 - y) @ s.T)))


def _sh_matrix(L_band, s):
    """Complex spherical harmonics Y_nm, 0 <= n < L_band, |m| <= n, at nodes s."""
    theta = np.arccos(np.clip(s[:, 2], -1, 1))
    phi = np.arctan2(s[:, 1], s[:, 0])
    cols = []
    for n in range(L_band):
        for m in range(-n, n + 1):
            cols.append(sph_harm_y(n, m, theta, phi))
    return np.stack(cols, axis=1)


def interpolation_matrix(Lc, Lp):
    """Band-limited resampling from the Lc grid to the Lp grid (degree < Lc);
    identity when the grids coincide."""
    if Lc == Lp:
        return np.eye(2 * Lc * Lc, dtype=np.complex128)
    sc, wc, _, _ = sphere_grid(Lc)
    sp, _, _, _ = sphere_grid(Lp)
    Yc = _sh_matrix(Lc, sc)
    Yp = _sh_matrix(Lc, sp)
    return Yp @ (Yc.conj().T * wc[None, :])


def anterpolation_matrix(Lp, Lc):
    """Weighted transpose of interpolation_matrix(Lc, Lp): parent grid -> child grid."""
    I = interpolation_matrix(Lc, Lp)
    _, wc, _, _ = sphere_grid(Lc)
    _, wp, _, _ = sphere_grid(Lp)
    return (I.T * wp[None, :]) / wc[:, None]


# --------------------------------------------------------------- matvec ---

class FMM:
    """Far-field operator of the multilevel FMM in plain steps."""

    def __init__(self, geom, k, p, levels, leaf_size, beta=None, gamma=None, tree=None, single=False,
                 level_rows=False):
        self.geom = geom
        self.k = k
        self.p = p
        self.gamma = coupling(k, gamma, p)
        N = geom["x"].shape[0]
        self.c = np.zeros(N, dtype=np.complex128) if beta is None else bc_factor(k, beta)
        self.tree = tree if tree is not None else build_tree(geom, levels, leaf_size, p["admissibility"])
        # levels above the first one with interaction pairs carry nothing:
        # no expansion there (length 0)
        nl = len(self.tree.levels)
        self.top = next((l for l, Lv in enumerate(self.tree.levels) if any(len(q) for q in Lv["il"])), nl - 1)
        self.L = [0 if l < self.top else
                  truncation_length(k, float(Lv["r"].max()), p, level_min_separation(Lv), single)
                  for l, Lv in enumerate(self.tree.levels)]
        self.grids = [sphere_grid(L) if L > 0 else None for L in self.L]
        # level_rows: the paper's variant -- every level aggregates from and
        # disaggregates to the elements with its own rows T(l), S(l)
        # (Sec. 3.3.4), no interpolation between levels
        self.level_rows = level_rows

    def signature_matrix(self, l, c_idx):
        """Rows nu, columns the elements of cluster c on level l: T_nu_j (c_j + ik s.n_j)."""
        Lv = self.tree.levels[l]
        g = self.geom
        els = Lv["groups"][c_idx]
        z = Lv["z"][c_idx]
        s, _, _, _ = self.grids[l]
        a, b, w = conical(self.p["t_order"])
        P0, P1, P2 = g["P0"][els], g["P1"][els], g["P2"][els]
        y = (P0[:, None, :] + a[None, :, None] * (P1 - P0)[:, None, :]
             + b[None, :, None] * (P2 - P0)[:, None, :])           # (ne, q, 3)
        ww = (2.0 * g["A"][els])[:, None] * w[None, :]              # (ne, q)
        ph = np.exp(1j * self.k * ((z[None, None, :] - y) @ s.T))  # (ne, q, nu)
        T = np.einsum("eq,eqv->ve", ww, ph)
        fac = self.c[els][None, :] + 1j * self.k * (s @ g["n"][els].T)
        return T * fac

    def distribution_matrix(self, l, c_idx):
        """Rows the elements of cluster c on level l, columns nu:
        ik/(16 pi^2) w_nu (1 - gamma ik s.n_i) exp(ik (x_i - z).s)."""
        Lv = self.tree.levels[l]
        g = self.geom
        els = Lv["groups"][c_idx]
        z = Lv["z"][c_idx]
        s, w, _, _ = self.grids[l]
        k = self.k
        S = np.exp(1j * k * ((g["x"][els] - z) @ s.T))
        fac = 1.0 - self.gamma * 1j * k * (g["n"][els] @ s.T)
        return (1j * k / (16 * math.pi ** 2)) * w[None, :] * fac * S

    def leaf_signature_matrix(self, c_idx):
        return self.signature_matrix(len(self.tree.levels) - 1, c_idx)

    def leaf_distribution_matrix(self, c_idx):
        return self.distribution_matrix(len(self.tree.levels) - 1, c_idx)

    def _translate(self, l, sig):
        Lv = self.tree.levels[l]
        s = self.grids[l][0]
        out = np.zeros_like(sig)
        pm = np.array([m for m in range(len(Lv["groups"])) for _ in Lv["il"][m]], dtype=np.int64)
        pn = np.array([n for m in range(len(Lv["groups"])) for n in Lv["il"][m]], dtype=np.int64)
        for b in range(0, pm.size, 2000):
            m_, n_ = pm[b:b + 2000], pn[b:b + 2000]
            D = translations(self.k, Lv["z"][m_] - Lv["z"][n_], s, self.L[l])
            np.add.at(out, m_, D * sig[n_])
        return out

    def _apply_level_rows(self, x):
        y = np.zeros(x.shape[0], dtype=np.complex128)
        for l in range(self.top, len(self.tree.levels)):
            Lv = self.tree.levels[l]
            if not any(len(q) for q in Lv["il"]):
                continue
            sig = np.stack([self.signature_matrix(l, c) @ x[g] for c, g in enumerate(Lv["groups"])])
            loc = self._translate(l, sig)
            for c, g in enumerate(Lv["groups"]):
                y[g] += self.distribution_matrix(l, c) @ loc[c]
        return y

    def apply(self, x):
        if self.level_rows:
            return self._apply_level_rows(x)
        tr = self.tree
        nl = len(tr.levels)
        k = self.k
        sig = [None] * nl
        leaf = tr.levels[-1]
        sig[-1] = np.stack([self.leaf_signature_matrix(c) @ x[g] for c, g in enumerate(leaf["groups"])])
        # upward: interpolate child signatures to the parent grid and shift
        for l in range(nl - 2, self.top - 1, -1):
            Lv, Cv = tr.levels[l], tr.levels[l + 1]
            I = interpolation_matrix(self.L[l + 1], self.L[l])
            sp = self.grids[l][0]
            out = np.zeros((len(Lv["groups"]), sp.shape[0]), dtype=np.complex128)
            for p in range(len(Lv["groups"])):
                for c in Lv["children"][p]:
                    shift = np.exp(1j * k * (sp @ (Lv["z"][p] - Cv["z"][c])))
                    out[p] += shift * (I @ sig[l + 1][c])
            sig[l] = out
        # translation on every level from the first one with pairs
        loc = [None] * self.top
        for l in range(self.top, nl):
            Lv = tr.levels[l]
            s = self.grids[l][0]
            out = np.zeros_like(sig[l])
            pm = np.array([m for m in range(len(Lv["groups"])) for _ in Lv["il"][m]], dtype=np.int64)
            pn = np.array([n for m in range(len(Lv["groups"])) for n in Lv["il"][m]], dtype=np.int64)
            for b in range(0, pm.size, 2000):
                m_, n_ = pm[b:b + 2000], pn[b:b + 2000]
                D = translations(k, Lv["z"][m_] - Lv["z"][n_], s, self.L[l])
                np.add.at(out, m_, D * sig[l][n_])
            loc.append(out)
        # downward: shift to the child centre and anterpolate
        for l in range(self.top, nl - 1):
            Lv, Cv = tr.levels[l], tr.levels[l + 1]
            Am = anterpolation_matrix(self.L[l], self.L[l + 1])
            sp = self.grids[l][0]
            for p in range(len(Lv["groups"])):
                for c in Lv["children"][p]:
                    shift = np.exp(1j * k * (sp @ (Cv["z"][c] - Lv["z"][p])))
                    loc[l + 1][c] += Am @ (shift * loc[l][p])
        y = np.zeros(x.shape[0], dtype=np.complex128)
        for c, g in enumerate(leaf["groups"]):
            y[g] += self.leaf_distribution_matrix(c) @ loc[-1][c]
        return y

    def near_mask_rows(self, rows):
        """Boolean (len(rows), N): True where (i, j) is a leaf near pair."""
        leaf = self.tree.levels[-1]
        N = self.geom["x"].shape[0]
        owner = np.empty(N, dtype=np.int64)
        for c, g in enumerate(leaf["groups"]):
            owner[g] = c
        mask = np.zeros((len(rows), N), dtype=bool)
        for r, i in enumerate(rows):
            for o in leaf["near"][owner[i]]:
                mask[r, leaf["groups"][o]] = True
        return mask
