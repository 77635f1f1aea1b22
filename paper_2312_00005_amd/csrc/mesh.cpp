// Host-side, frequency-independent setup: element geometry, the cluster tree
// with near and interaction lists, and the near-field quadrature plan.
//
// Geometry (Sec. 2.2-2.3, mesh appendix): flat triangles and plane
// quadrilaterals, collocation node = vertex mean, unit normal from the
// counter-clockwise vertex order, area.
//
// Cluster tree (Sec. 3.3.2-3.3.4), as read here:
//  * A group of elements is split by putting a box around its vertices and
//    cutting every axis into max(1, floor(extent/edge + 1/2)) equal slabs; an
//    element belongs to the sub-box that holds its centroid; empty boxes are
//    dropped; sub-boxes are ordered lexicographically (x, then y, then z).
//  * A cluster's midpoint is the mean over the vertex incidences of its
//    elements; its radius is the largest vertex distance from the midpoint.
//  * Small clusters -- radius below half the mean radius of the group, or
//    fewer than leaf_size/4 elements -- are merged into the nearest (by
//    midpoint) non-small cluster of the same group.
//  * The root level splits the whole mesh with edge e_r; level l (root = 1)
//    splits every cluster of level l-1 with edge e_r / 2^(l-1).  All leaves
//    are on the last level.  With e_r = 0 the leaf edge is
//    sqrt(leaf_size * mean element area) and e_r = leaf edge * 2^(levels-1).
//  * Two clusters are far if |z_i - z_j| > a (r_i + r_j) (Eq. (Farfieldcond)
//    with a parameter a).  On the root level every far pair is in the
//    interaction list; on level l > 1 the candidates of a cluster are the
//    children of its parent's near clusters, far ones form its interaction
//    list and the rest its near list.  Near pairs exist on the leaf level.
//
// Near-field plan (Sec. 3.1.3-3.1.4): for every near pair (i, j), i != j, and
// every integration triangle of j (the element itself, or the two halves of
// a quadrilateral, each with its own midpoint and area), the triangle is
// split into four through its edge midpoints while r~ = |x_i - mid| / sqrt(A)
// < ratio; otherwise the order m is the smallest
// with the three a-priori estimates below eps; an order above m_max is capped
// or, with split_on_cap, split once more.  More than max_subdiv nested splits
// is an error naming the element.
#include <algorithm>
#include <cstdio>
#include <numeric>

#include "common.h"

namespace bem {

Geometry build_geometry(const double* xyz, int64_t n_nodes, const int32_t* el,
                        int64_t n_el, const std::vector<int64_t>& perm) {
  Geometry g;
  g.N = n_el;
  g.f.assign(size_t(G_NFIELDS) * n_el, 0.0);
  std::vector<int64_t> quads;  // tree positions of the quadrilaterals
  for (int64_t t = 0; t < n_el; ++t) {
    int64_t e = perm[t];
    const int32_t* v = el + 4 * e;
    const int nv = v[3] >= 0 ? 4 : 3;
    for (int c = 0; c < nv; ++c)
      if (v[c] < 0 || v[c] >= n_nodes)
        throw Error(BEM_E_ARG, "element " + std::to_string(e) + " has a node index out of range", e);
    const double* a = xyz + 3 * v[0];
    const double* b = xyz + 3 * v[1];
    const double* c = xyz + 3 * v[2];
    if (nv == 3) {
      double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
      double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
      double nrm = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      if (!(nrm > 0.0) || !std::isfinite(nrm))
        throw Error(BEM_E_MESH, "triangle " + std::to_string(e) + " has zero or invalid area", e);
      for (int d = 0; d < 3; ++d) {
        g.at(G_P0X + d, t) = a[d];
        g.at(G_P1X + d, t) = b[d];
        g.at(G_P2X + d, t) = c[d];
        g.at(G_NX + d, t) = cr[d] / nrm;
        g.at(G_CX + d, t) = (a[d] + b[d] + c[d]) / 3.0;
      }
      g.at(G_AREA, t) = 0.5 * nrm;
      continue;
    }
    const double* q = xyz + 3 * v[3];
    double d1[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double d2[3] = {q[0] - b[0], q[1] - b[1], q[2] - b[2]};
    double cr[3] = {d1[1] * d2[2] - d1[2] * d2[1], d1[2] * d2[0] - d1[0] * d2[2], d1[0] * d2[1] - d1[1] * d2[0]};
    double nrm = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    if (!(nrm > 0.0) || !std::isfinite(nrm))
      throw Error(BEM_E_MESH, "quadrilateral " + std::to_string(e) + " has zero or invalid area", e);
    double n[3] = {cr[0] / nrm, cr[1] / nrm, cr[2] / nrm}, mid[3];
    for (int d = 0; d < 3; ++d) mid[d] = 0.25 * (a[d] + b[d] + c[d] + q[d]);
    // plane: every vertex within 1e-8 of the longer diagonal from the mean plane
    const double diag = std::sqrt(std::max(d1[0] * d1[0] + d1[1] * d1[1] + d1[2] * d1[2],
                                           d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2]));
    for (const double* p : {a, b, c, q}) {
      const double off = (p[0] - mid[0]) * n[0] + (p[1] - mid[1]) * n[1] + (p[2] - mid[2]) * n[2];
      if (std::fabs(off) > 1e-8 * diag)
        throw Error(BEM_E_MESH, "quadrilateral " + std::to_string(e) + " is not plane", e);
    }
    // convex and counter-clockwise about n: every corner turns the same way
    const double* P[4] = {a, b, c, q};
    for (int k = 0; k < 4; ++k) {
      const double* p0 = P[k];
      const double* p1 = P[(k + 1) % 4];
      const double* p2 = P[(k + 2) % 4];
      double u[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
      double w[3] = {p2[0] - p1[0], p2[1] - p1[1], p2[2] - p1[2]};
      double x[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
      if (!(x[0] * n[0] + x[1] * n[1] + x[2] * n[2] > 0.0))
        throw Error(BEM_E_MESH, "quadrilateral " + std::to_string(e) + " is not convex", e);
    }
    for (int d = 0; d < 3; ++d) {
      g.at(G_P0X + d, t) = a[d];
      g.at(G_P1X + d, t) = b[d];
      g.at(G_P2X + d, t) = c[d];
      g.at(G_NX + d, t) = n[d];
      g.at(G_CX + d, t) = mid[d];
    }
    g.at(G_AREA, t) = 0.5 * nrm;
    quads.push_back(t);
  }
  if (quads.empty()) return g;
  g.nq = (int64_t)quads.size();
  const int64_t nh = 2 * g.nq;
  g.qidx.assign(n_el, -1);
  g.hown.resize(nh);
  g.hq.assign(size_t(G_NFIELDS) * nh, 0.0);
  for (int64_t qi = 0; qi < g.nq; ++qi) {
    const int64_t t = quads[qi];
    g.qidx[t] = qi;
    const int32_t* v = el + 4 * perm[t];
    const int32_t tri[2][3] = {{v[0], v[1], v[2]}, {v[0], v[2], v[3]}};
    for (int h = 0; h < 2; ++h) {
      const int64_t r = 2 * qi + h;
      g.hown[r] = t;
      const double* a = xyz + 3 * tri[h][0];
      const double* b = xyz + 3 * tri[h][1];
      const double* c = xyz + 3 * tri[h][2];
      double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
      double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
      const double nrm = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      for (int d = 0; d < 3; ++d) {
        g.hq[(G_P0X + d) * nh + r] = a[d];
        g.hq[(G_P1X + d) * nh + r] = b[d];
        g.hq[(G_P2X + d) * nh + r] = c[d];
        g.hq[(G_NX + d) * nh + r] = g.at(G_NX + d, t);
        g.hq[(G_CX + d) * nh + r] = (a[d] + b[d] + c[d]) / 3.0;
      }
      g.hq[G_AREA * nh + r] = 0.5 * nrm;
    }
  }
  return g;
}

namespace {

struct Group {
  std::vector<int64_t> e;  // ascending caller indices
  double z[3] = {0, 0, 0};
  double r = 0;
};

void group_stats(const Geometry& g, Group& G) {
  double s[3] = {0, 0, 0};
  double cnt = 0.0;
  for (int64_t e : G.e) {
    const int nv = g.nv(e);
    for (int v = 0; v < nv; ++v)
      for (int d = 0; d < 3; ++d) s[d] += g.vtx(v, d, e);
    cnt += nv;
  }
  for (int d = 0; d < 3; ++d) G.z[d] = s[d] / cnt;
  double r2 = 0.0;
  for (int64_t e : G.e)
    for (int v = 0; v < g.nv(e); ++v) {
      double dx = g.vtx(v, 0, e) - G.z[0];
      double dy = g.vtx(v, 1, e) - G.z[1];
      double dz = g.vtx(v, 2, e) - G.z[2];
      double q = dx * dx + dy * dy + dz * dz;
      if (q > r2) r2 = q;
    }
  G.r = std::sqrt(r2);
}

std::vector<Group> split_group(const Geometry& g, const std::vector<int64_t>& elems, double edge) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t e : elems)
    for (int v = 0; v < g.nv(e); ++v)
      for (int d = 0; d < 3; ++d) {
        double c = g.vtx(v, d, e);
        lo[d] = std::min(lo[d], c);
        hi[d] = std::max(hi[d], c);
      }
  int64_t n[3];
  double ext[3];
  for (int d = 0; d < 3; ++d) {
    ext[d] = hi[d] - lo[d];
    n[d] = std::max<int64_t>(1, (int64_t)std::floor(ext[d] / edge + 0.5));
  }
  std::vector<std::pair<int64_t, int64_t>> keyed;
  keyed.reserve(elems.size());
  for (int64_t e : elems) {
    int64_t idx[3];
    for (int d = 0; d < 3; ++d) {
      if (n[d] == 1) { idx[d] = 0; continue; }
      double t = (g.at(G_CX + d, e) - lo[d]) * double(n[d]) / ext[d];
      int64_t q = (int64_t)std::floor(t);
      idx[d] = std::min<int64_t>(n[d] - 1, std::max<int64_t>(0, q));
    }
    keyed.push_back({(idx[0] * n[1] + idx[1]) * n[2] + idx[2], e});
  }
  std::stable_sort(keyed.begin(), keyed.end(),
                   [](const std::pair<int64_t, int64_t>& a, const std::pair<int64_t, int64_t>& b) {
                     return a.first < b.first;
                   });
  std::vector<Group> out;
  for (size_t i = 0; i < keyed.size();) {
    size_t j = i;
    Group G;
    while (j < keyed.size() && keyed[j].first == keyed[i].first) G.e.push_back(keyed[j++].second);
    out.push_back(std::move(G));
    i = j;
  }
  for (auto& G : out) group_stats(g, G);
  return out;
}

std::vector<Group> merge_small(const Geometry& g, std::vector<Group> grp, int leaf_size) {
  size_t ng = grp.size();
  if (ng <= 1) return grp;
  double rsum = 0.0;
  for (auto& G : grp) rsum += G.r;
  double rmean = rsum / double(ng);
  int64_t nmin = std::max(1, leaf_size / 4);
  std::vector<char> small(ng);
  size_t n_small = 0;
  for (size_t i = 0; i < ng; ++i) {
    small[i] = (grp[i].r < 0.5 * rmean) || ((int64_t)grp[i].e.size() < nmin);
    n_small += small[i];
  }
  if (n_small == 0 || n_small == ng) return grp;
  std::vector<int64_t> target(ng, -1);
  for (size_t i = 0; i < ng; ++i) {
    if (!small[i]) continue;
    double best = INFINITY;
    int64_t bi = -1;
    for (size_t j = 0; j < ng; ++j) {
      if (small[j]) continue;
      double dx = grp[i].z[0] - grp[j].z[0], dy = grp[i].z[1] - grp[j].z[1], dz = grp[i].z[2] - grp[j].z[2];
      double d2 = dx * dx + dy * dy + dz * dz;
      if (d2 < best) { best = d2; bi = (int64_t)j; }
    }
    target[i] = bi;
  }
  std::vector<Group> out;
  for (size_t j = 0; j < ng; ++j) {
    if (small[j]) continue;
    Group G;
    G.e = grp[j].e;
    for (size_t i = 0; i < ng; ++i)
      if (small[i] && target[i] == (int64_t)j) G.e.insert(G.e.end(), grp[i].e.begin(), grp[i].e.end());
    std::sort(G.e.begin(), G.e.end());
    group_stats(g, G);
    out.push_back(std::move(G));
  }
  return out;
}

bool is_far(const Level& L, int64_t a, int64_t b, double adm) {
  double dx = L.z[3 * a] - L.z[3 * b], dy = L.z[3 * a + 1] - L.z[3 * b + 1], dz = L.z[3 * a + 2] - L.z[3 * b + 2];
  double d2 = dx * dx + dy * dy + dz * dz;
  double lim = adm * (L.r[a] + L.r[b]);
  return d2 > lim * lim;
}

}  // namespace

Tree build_tree(const Geometry& gc, int levels, double root_edge, int leaf_size, double adm) {
  if (levels < 1 || levels > 16) throw Error(BEM_E_ARG, "levels must be in [1, 16]");
  int64_t N = gc.N;
  if (root_edge <= 0.0) {
    double asum = 0.0;
    for (int64_t e = 0; e < N; ++e) asum += gc.at(G_AREA, e);
    double leaf_edge = std::sqrt(double(leaf_size) * (asum / double(N)));
    root_edge = leaf_edge * std::ldexp(1.0, levels - 1);
  }
  std::vector<int64_t> all(N);
  std::iota(all.begin(), all.end(), 0);
  std::vector<std::vector<Group>> lvg(levels);
  std::vector<std::vector<int64_t>> parent(levels);
  lvg[0] = merge_small(gc, split_group(gc, all, root_edge), leaf_size);
  parent[0].assign(lvg[0].size(), -1);
  for (int l = 1; l < levels; ++l) {
    double edge = root_edge / std::ldexp(1.0, l);
    for (size_t p = 0; p < lvg[l - 1].size(); ++p) {
      auto ch = merge_small(gc, split_group(gc, lvg[l - 1][p].e, edge), leaf_size);
      for (auto& c : ch) {
        lvg[l].push_back(std::move(c));
        parent[l].push_back((int64_t)p);
      }
    }
  }
  Tree T;
  T.lv.resize(levels);
  // tree order: concatenation of leaves
  for (auto& G : lvg[levels - 1]) T.perm.insert(T.perm.end(), G.e.begin(), G.e.end());
  T.inv.assign(N, -1);
  for (int64_t t = 0; t < N; ++t) T.inv[T.perm[t]] = t;
  for (int l = levels - 1; l >= 0; --l) {
    Level& L = T.lv[l];
    L.nc = (int64_t)lvg[l].size();
    L.z.resize(3 * L.nc);
    L.r.resize(L.nc);
    L.ebeg.resize(L.nc);
    L.eend.resize(L.nc);
    L.parent = parent[l];
    for (int64_t c = 0; c < L.nc; ++c) {
      for (int d = 0; d < 3; ++d) L.z[3 * c + d] = lvg[l][c].z[d];
      L.r[c] = lvg[l][c].r;
    }
    if (l == levels - 1) {
      int64_t pos = 0;
      for (int64_t c = 0; c < L.nc; ++c) {
        L.ebeg[c] = pos;
        pos += (int64_t)lvg[l][c].e.size();
        L.eend[c] = pos;
      }
    } else {
      Level& C = T.lv[l + 1];
      L.cbeg.assign(L.nc, -1);
      L.cend.assign(L.nc, -1);
      for (int64_t c = 0; c < C.nc; ++c) {
        int64_t p = C.parent[c];
        if (L.cbeg[p] < 0) L.cbeg[p] = c;
        L.cend[p] = c + 1;
      }
      for (int64_t p = 0; p < L.nc; ++p) {
        L.ebeg[p] = C.ebeg[L.cbeg[p]];
        L.eend[p] = C.eend[L.cend[p] - 1];
      }
    }
  }
  // near and interaction lists
  for (int l = 0; l < levels; ++l) {
    Level& L = T.lv[l];
    L.il_off.assign(L.nc + 1, 0);
    L.nr_off.assign(L.nc + 1, 0);
    L.il.clear();
    L.nr.clear();
    for (int64_t c = 0; c < L.nc; ++c) {
      if (l == 0) {
        for (int64_t o = 0; o < L.nc; ++o) (is_far(L, c, o, adm) ? L.il : L.nr).push_back(o);
      } else {
        const Level& P = T.lv[l - 1];
        int64_t p = L.parent[c];
        for (int64_t t = P.nr_off[p]; t < P.nr_off[p + 1]; ++t) {
          int64_t q = P.nr[t];
          for (int64_t o = P.cbeg[q]; o < P.cend[q]; ++o) (is_far(L, c, o, adm) ? L.il : L.nr).push_back(o);
        }
      }
      L.il_off[c + 1] = (int64_t)L.il.size();
      L.nr_off[c + 1] = (int64_t)L.nr.size();
    }
  }
  return T;
}

namespace {

// Rule order of a (sub-)element (Sec. 3.1.4): the smallest m whose three
// a-priori estimates 32 q^(2m+1), 64 (2m+1) q^(2m+2), 128 (m+1)(2m+1) q^(2m+3),
// q = 1/(2 r~), are all below eps.  Each estimate grows with q, so order m
// holds iff q is below the smallest root of the three, i.e. iff r~ > th[m]:
// the table gives the order without powers, and within 1e-12 (relative) of a
// threshold the estimates themselves decide, so the choice is the
// estimates', bit for bit.
struct OrderTable {
  double th[65];
  explicit OrderTable(double eps) {
    for (int m = 1; m <= 64; ++m) {
      const double q1 = std::pow(eps / 32.0, 1.0 / (2 * m + 1));
      const double q2 = std::pow(eps / (64.0 * (2 * m + 1)), 1.0 / (2 * m + 2));
      const double q3 = std::pow(eps / (128.0 * (m + 1) * (2 * m + 1)), 1.0 / (2 * m + 3));
      th[m] = 1.0 / (2.0 * std::min(q1, std::min(q2, q3)));
    }
    th[0] = 0.0;
  }
};

bool order_holds(double rt, double eps, int m) {
  const double q = 1.0 / (2.0 * rt);
  const double eg = 32.0 * std::pow(q, double(2 * m + 1));
  const double eh = 64.0 * double(2 * m + 1) * std::pow(q, double(2 * m + 2));
  const double ee = 128.0 * double(m + 1) * double(2 * m + 1) * std::pow(q, double(2 * m + 3));
  return eg < eps && eh < eps && ee < eps;
}

int estimator_order_fast(double rt, double eps, const OrderTable& T) {
  for (int m = 1; m <= 64; ++m) {
    const double t = T.th[m];
    if (rt > t * (1.0 + 1e-12)) return m;
    if (rt >= t * (1.0 - 1e-12) && order_holds(rt, eps, m)) return m;
  }
  return 64;
}

struct PlanCtx {
  const QuadParams* q;
  const OrderTable* ot;
  double x[3];
  int64_t j;
  std::vector<uint64_t>* out;
  int64_t points;
  int max_m;
  int64_t bad;
};

void plan_rec(PlanCtx& C, const double* v0, const double* v1, const double* v2, double area,
              int depth, uint64_t path) {
  double mid[3], d[3];
  for (int c = 0; c < 3; ++c) {
    mid[c] = (v0[c] + v1[c] + v2[c]) / 3.0;
    d[c] = C.x[c] - mid[c];
  }
  double rt = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) / std::sqrt(area);
  bool split = rt < C.q->ratio;
  int m = 1;
  if (!split) {
    m = estimator_order_fast(rt, C.q->eps, *C.ot);
    if (m > C.q->m_max) {
      if (C.q->split_on_cap) split = true;
      else m = C.q->m_max;
    }
  }
  if (split) {
    if (depth >= C.q->max_subdiv) {
      if (C.bad < 0) C.bad = C.j;
      return;
    }
    double m01[3], m12[3], m20[3];
    for (int c = 0; c < 3; ++c) {
      m01[c] = 0.5 * (v0[c] + v1[c]);
      m12[c] = 0.5 * (v1[c] + v2[c]);
      m20[c] = 0.5 * (v2[c] + v0[c]);
    }
    double a4 = area * 0.25;
    plan_rec(C, v0, m01, m20, a4, depth + 1, path | (uint64_t(0) << (2 * depth)));
    plan_rec(C, v1, m12, m01, a4, depth + 1, path | (uint64_t(1) << (2 * depth)));
    plan_rec(C, v2, m20, m12, a4, depth + 1, path | (uint64_t(2) << (2 * depth)));
    plan_rec(C, m01, m12, m20, a4, depth + 1, path | (uint64_t(3) << (2 * depth)));
    return;
  }
  uint64_t item = uint64_t(C.j) | (uint64_t(m - 1) << 26) | (uint64_t(depth) << 29) | (path << 33);
  C.out->push_back(item);
  C.points += int64_t(m) * m;
  if (m > C.max_m) C.max_m = m;
}

}  // namespace

NearPlan build_near_plan(const Geometry& g, const QuadParams& q,
                         const std::vector<int64_t>& tgt_src_off,
                         const std::vector<int64_t>& src_beg,
                         const std::vector<int64_t>& src_end,
                         const std::vector<int64_t>& tgt_group) {
  if (q.max_subdiv > 15) throw Error(BEM_E_ARG, "max_subdiv above 15 is not supported");
  if (q.m_max > 8 || q.m_max < 1) throw Error(BEM_E_ARG, "quad_m_max must be in [1, 8]");
  int64_t N = g.N;
  const int64_t nh = 2 * g.nq;
  if (N + nh >= (int64_t(1) << 26)) throw Error(BEM_E_ARG, "too many elements for the packed plan");
  std::vector<std::vector<uint64_t>> per(N);
  std::vector<int64_t> pts(N, 0), npairs(N, 0), bad(N, -1);
  std::vector<int> mm(N, 1);
  const OrderTable ot(q.eps);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < N; ++t) {
    PlanCtx C;
    C.q = &q;
    C.ot = &ot;
    for (int c = 0; c < 3; ++c) C.x[c] = g.at(G_CX + c, t);
    C.out = &per[t];
    C.points = 0;
    C.max_m = 1;
    C.bad = -1;
    int64_t grp = tgt_group[t];
    for (int64_t s = tgt_src_off[grp]; s < tgt_src_off[grp + 1]; ++s) {
      for (int64_t j = src_beg[s]; j < src_end[s]; ++j) {
        ++npairs[t];
        if (j == t) continue;
        if (!g.is_quad(j)) {
          C.j = j;
          double v0[3] = {g.at(G_P0X, j), g.at(G_P0Y, j), g.at(G_P0Z, j)};
          double v1[3] = {g.at(G_P1X, j), g.at(G_P1Y, j), g.at(G_P1Z, j)};
          double v2[3] = {g.at(G_P2X, j), g.at(G_P2Y, j), g.at(G_P2Z, j)};
          plan_rec(C, v0, v1, v2, g.at(G_AREA, j), 0, 0);
          continue;
        }
        // a quadrilateral: its two integration triangles, each with its own r~
        for (int h = 0; h < 2; ++h) {
          const int64_t r = 2 * g.qidx[j] + h;
          C.j = N + r;
          double v[3][3];
          for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) v[a][d] = g.hq[(G_P0X + 3 * a + d) * nh + r];
          plan_rec(C, v[0], v[1], v[2], g.hq[G_AREA * nh + r], 0, 0);
        }
      }
    }
    // group items by order so that a wavefront mostly runs one rule
    std::stable_sort(per[t].begin(), per[t].end(), [](uint64_t a, uint64_t b) {
      return ((a >> 26) & 7) < ((b >> 26) & 7);
    });
    pts[t] = C.points;
    mm[t] = C.max_m;
    bad[t] = C.bad;
  }
  for (int64_t t = 0; t < N; ++t)
    if (bad[t] >= 0) {
      const int64_t e = g.owner(bad[t]);
      throw Error(BEM_E_MESH, "more than max_subdiv nested subdivisions (element at tree position " +
                                  std::to_string(e) + ")", e);
    }
  NearPlan P;
  P.off.assign(N + 1, 0);
  for (int64_t t = 0; t < N; ++t) {
    P.off[t + 1] = P.off[t] + (int64_t)per[t].size();
    P.points += pts[t];
    P.pairs += npairs[t];
    P.max_m = std::max(P.max_m, mm[t]);
  }
  P.items.resize(P.off[N]);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < N; ++t) std::copy(per[t].begin(), per[t].end(), P.items.begin() + P.off[t]);
  build_segments(P, N);
  return P;
}

void build_segments(NearPlan& P, int64_t N) {
  const int S = 9;
  P.seg.assign((size_t)N * S, 0);
  int64_t unsorted = 0;
#pragma omp parallel for schedule(static) reduction(+ : unsorted)
  for (int64_t t = 0; t < N; ++t) {
    int64_t q = P.off[t];
    for (int mc = 0; mc < 8; ++mc) {
      P.seg[(size_t)t * S + mc] = q;
      while (q < P.off[t + 1] && (int)((P.items[q] >> 26) & 7u) == mc) ++q;
    }
    P.seg[(size_t)t * S + 8] = P.off[t + 1];
    if (q != P.off[t + 1]) ++unsorted;
  }
  if (unsorted) throw Error(BEM_E_STATE, "near-field items are not sorted by rule order");
}

}  // namespace bem
