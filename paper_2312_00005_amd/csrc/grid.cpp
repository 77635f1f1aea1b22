// Evaluation grid (the paper's evaluation points, output appendix): pressure
// at many field points with the far part from the FMM.
//
// The points are grouped into point clusters by boxes whose half diagonal is
// the largest leaf-cluster radius of the mesh, so that every point cluster is
// no larger than a leaf cluster and the leaf level's expansion length holds
// for its pairs.  A (point cluster P, leaf cluster C) pair is far when
// |z_P - z_C| > a (r_P + r_C) with the mesh's admissibility a (Eq.
// (Farfieldcond)) and the translation operator passes the stability test of
// the FP64 lengths; all other pairs are integrated directly.  Far part, from
// the expansion of Eq. (FMMBase) about z_P and z_C on the leaf grid:
//   Sig_C(nu) = sum_{j in C} T_j(nu) (ik (s.n_j) p_j + v_j),
//   Loc_P(nu) = sum_{C far} D(z_P - z_C, s_nu) Sig_C(nu),
//   p_far(x)  = -(ik / 16 pi^2) sum_nu w_nu exp(ik (x - z_P).s_nu) Loc_P(nu),
// the expansion of sum_j (I^H_j(x) p_j - I^G_j(x) v_j) (a derivative in y
// multiplies the outgoing plane wave by -ik s.n_j).  The translation values
// are evaluated on the fly from their Legendre series, nothing of size
// pairs x nodes is stored.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <memory>

#include "fmm.h"
#include "guard.h"
#include "state.h"

using namespace bem;

struct bem_grid {
  bem_mesh* m = nullptr;
  int64_t npts = 0;
  std::vector<int64_t> order;   // cluster-order position -> caller index
  std::vector<double> pts;      // cluster order, 3 per point
  std::vector<int64_t> pc;      // point -> point cluster
  std::vector<double> zp, rp;   // point clusters: centre (3), radius
  int64_t npc = 0;
  DevBuf<double> d_pts, d_zp, d_zc;
  DevBuf<int64_t> d_order, d_pc;
  // split of the current problem
  uint64_t stamp = ~uint64_t(0);
  int L = -1;
  int64_t npairs = 0, near_elems = 0;
  DevBuf<int64_t> d_far_off, d_pair_p, d_pair_c, d_near_off, d_near_beg, d_near_end;
  DevBuf<double2> d_coef;
  DevBuf<double> d_dir;
  DevBuf<double2> d_sigA, d_sigB, d_loc, d_p, d_v, d_out, d_pinc;
  DevBuf<int64_t> d_err;
};

namespace {

void build_points(bem_grid* g, const double* xyz) {
  const Level& leaf = g->m->tree.lv.back();
  double rmax = 0.0;
  for (double r : leaf.r) rmax = std::max(rmax, r);
  if (!(rmax > 0.0)) throw Error(BEM_E_STATE, "the mesh's leaf clusters have no extent");
  const double edge = 2.0 * rmax / std::sqrt(3.0);
  double lo[3] = {xyz[0], xyz[1], xyz[2]};
  for (int64_t i = 0; i < g->npts; ++i)
    for (int d = 0; d < 3; ++d) lo[d] = std::min(lo[d], xyz[3 * i + d]);
  std::vector<std::array<int64_t, 3>> box(g->npts);
  for (int64_t i = 0; i < g->npts; ++i)
    for (int d = 0; d < 3; ++d) box[i][d] = (int64_t)std::floor((xyz[3 * i + d] - lo[d]) / edge);
  g->order.resize(g->npts);
  for (int64_t i = 0; i < g->npts; ++i) g->order[i] = i;
  std::stable_sort(g->order.begin(), g->order.end(), [&](int64_t a, int64_t b) { return box[a] < box[b]; });
  g->pts.resize(3 * g->npts);
  g->pc.resize(g->npts);
  g->zp.clear();
  g->rp.clear();
  int64_t c = -1;
  for (int64_t t = 0; t < g->npts; ++t) {
    const int64_t i = g->order[t];
    if (t == 0 || box[i] != box[g->order[t - 1]]) {
      ++c;
      for (int d = 0; d < 3; ++d) g->zp.push_back(lo[d] + (box[i][d] + 0.5) * edge);
      g->rp.push_back(0.0);
    }
    g->pc[t] = c;
    double r2 = 0.0;
    for (int d = 0; d < 3; ++d) {
      g->pts[3 * t + d] = xyz[3 * i + d];
      const double dd = xyz[3 * i + d] - g->zp[3 * c + d];
      r2 += dd * dd;
    }
    g->rp[c] = std::max(g->rp[c], std::sqrt(r2));
  }
  g->npc = c + 1;
}

// far / near lists of the current problem (the stability test depends on k)
void build_split(bem_grid* g, hipStream_t s) {
  bem_mesh* m = g->m;
  const FmmLeafView v = fmm_leaf_view(m);
  const Level& leaf = m->tree.lv.back();
  const double a = m->opt.admissibility;
  std::vector<int64_t> far_off(g->npc + 1, 0), pp, pcl, near_off(g->npc + 1, 0), nb, ne;
  int64_t nel = 0;
  for (int64_t P = 0; P < g->npc; ++P) {
    for (int64_t C = 0; C < leaf.nc; ++C) {
      double X2 = 0.0;
      for (int d = 0; d < 3; ++d) {
        const double dd = g->zp[3 * P + d] - leaf.z[3 * C + d];
        X2 += dd * dd;
      }
      const double X = std::sqrt(X2);
      if (X > a * (g->rp[P] + leaf.r[C]) && fmm_leaf_pair_stable(m, v.L, X)) {
        pp.push_back(P);
        pcl.push_back(C);
      } else {
        nb.push_back(leaf.ebeg[C]);
        ne.push_back(leaf.eend[C]);
        nel += leaf.eend[C] - leaf.ebeg[C];
      }
    }
    far_off[P + 1] = (int64_t)pp.size();
    near_off[P + 1] = (int64_t)nb.size();
  }
  g->npairs = (int64_t)pp.size();
  g->near_elems = nel;
  if (pp.empty()) {
    pp.push_back(0);
    pcl.push_back(0);
  }
  if (nb.empty()) {
    nb.push_back(0);
    ne.push_back(0);
  }
  g->d_far_off.upload(far_off, s);
  g->d_pair_p.upload(pp, s);
  g->d_pair_c.upload(pcl, s);
  g->d_near_off.upload(near_off, s);
  g->d_near_beg.upload(nb, s);
  g->d_near_end.upload(ne, s);
  g->d_zc.upload(leaf.z, s);
  g->L = v.L;
  g->d_coef.alloc((size_t)std::max<int64_t>(1, g->npairs) * (v.L + 1));
  g->d_dir.alloc((size_t)std::max<int64_t>(1, g->npairs) * 3);
  launch_grid_coef(g->npairs, g->d_pair_p.p, g->d_pair_c.p, g->d_zp.p, g->d_zc.p, m->k, v.L, g->d_coef.p,
                   g->d_dir.p, s);
  g->d_sigA.alloc((size_t)v.nc * v.nu);
  g->d_sigB.alloc((size_t)v.nc * v.nu);
  g->d_loc.alloc((size_t)g->npc * v.nu);
  g->stamp = m->problem_stamp;
}

}  // namespace

extern "C" {

bem_status bem_grid_create(bem_mesh* m, int64_t n_pts, const double* pts, bem_grid** out) {
  return guarded([&]() -> bem_status {
    if (!m || !out || n_pts < 1 || !pts) return fail(BEM_E_ARG, "NULL argument or no points");
    *out = nullptr;
    if (!m->fmm || m->far_direct || m->far_direct64)
      return fail(BEM_E_STATE, "the evaluation grid needs a mesh with the FP64 FMM (far_direct = 0)");
    for (int64_t i = 0; i < 3 * n_pts; ++i)
      if (!std::isfinite(pts[i])) return fail(BEM_E_ARG, "non-finite point coordinate");
    auto g = std::make_unique<bem_grid>();
    g->m = m;
    g->npts = n_pts;
    build_points(g.get(), pts);
    hipStream_t s = nullptr;
    g->d_pts.upload(g->pts, s);
    g->d_zp.upload(g->zp, s);
    g->d_order.upload(g->order, s);
    g->d_pc.upload(g->pc, s);
    g->d_p.alloc(m->N);
    g->d_v.alloc(m->N);
    g->d_out.alloc(n_pts);
    g->d_pinc.alloc(n_pts);
    g->d_err.alloc(1);
    *out = g.release();
    return BEM_OK;
  });
}

bem_status bem_grid_eval(bem_grid* g, const bem_c128* p_surf, const bem_c128* dpdn_surf, const bem_c128* p_inc,
                         bem_c128* p_out, double* energy, void* stream) {
  return guarded([&]() -> bem_status {
    if (!g || !p_surf || !p_out) return fail(BEM_E_ARG, "NULL argument");
    bem_mesh* m = g->m;
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    if (m->has_pres && !dpdn_surf)
      return fail(BEM_E_ARG, "the mesh has PRES elements: dpdn_surf is required");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (g->stamp != m->problem_stamp) build_split(g, s);
    const FmmLeafView v = fmm_leaf_view(m);
    launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(p_surf), g->d_p.p, s);
    if (dpdn_surf)
      launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(dpdn_surf), g->d_v.p, s);
    else
      launch_cmul(m->N, m->have_beta ? m->d_cfac.p : nullptr, g->d_p.p, g->d_v.p, s);
    fmm_leaf_aggregate(m, g->d_p.p, true, g->d_sigA.p, s);
    fmm_leaf_aggregate(m, g->d_v.p, false, g->d_sigB.p, s);
    launch_grid_translate(g->npc, g->d_far_off.p, g->d_pair_c.p, g->d_coef.p, g->d_dir.p, g->L, v.nu, v.s,
                          g->d_sigA.p, g->d_sigB.p, g->d_loc.p, s);
    if (p_inc)
      launch_gather(g->npts, g->d_order.p, reinterpret_cast<const double2*>(p_inc), g->d_pinc.p, s);
    launch_fill_i64(1, -1, g->d_err.p, s);
    FieldArgs A = field_args(m, g->npts, 0);
    launch_grid_eval(A, g->d_pts.p, g->d_pc.p, g->d_zp.p, v.nu, v.s, v.w, g->d_loc.p, g->d_near_off.p,
                     g->d_near_beg.p, g->d_near_end.p, g->d_p.p, g->d_v.p, p_inc ? g->d_pinc.p : nullptr,
                     g->d_out.p, g->d_err.p, s);
    launch_scatter(g->npts, g->d_order.p, g->d_out.p, reinterpret_cast<double2*>(p_out), s);
    if (energy) launch_energy(g->npts, reinterpret_cast<const double2*>(p_out), energy, s);
    BEM_HIP(hipGetLastError());
    check_field_error(m, g->d_err.p, s);
    return BEM_OK;
  });
}

bem_status bem_grid_stats(const bem_grid* g, int64_t* point_clusters, int64_t* far_pairs, int64_t* near_elements) {
  return guarded([&]() -> bem_status {
    if (!g) return fail(BEM_E_ARG, "grid is NULL");
    if (point_clusters) *point_clusters = g->npc;
    if (far_pairs) *far_pairs = g->npairs;
    if (near_elements) *near_elements = g->near_elems;
    return BEM_OK;
  });
}

void bem_grid_destroy(bem_grid* g) { delete g; }

}  // extern "C"
