// C ABI entry points (include/bemfmm.h).  Every entry point catches
// exceptions and turns them into a status code plus a thread-local message.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "guard.h"
#include "fmm.h"
#include "state.h"

using namespace bem;

namespace {

thread_local std::string g_last_error;

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

void set_paper(bem_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->use_fmm = 1;
  o->levels = 0;
  o->leaf_size = 25;
  o->root_box_edge = 0.0;
  o->admissibility = 2.0 / std::sqrt(3.0);
  o->l_mode = 0;
  o->l_factor = 1.8;
  o->l_min = 8;
  o->l_eps = 1e-3;
  o->t_order = 4;
  o->quad_eps = 1e-3;
  o->quad_eps_mixed = 1e-3;
  o->quad_m_max = 6;
  o->quad_split_on_cap = 0;
  o->subdiv_ratio = 1.3;
  o->max_subdiv = 15;
  o->self_n = 4;
  o->edge_parts = 4;
  o->edge_gauss = 3;
  o->precision = BEM_PREC_FP64;
  o->gmres_restart = 100;
  o->gmres_maxit = 250;
  o->gmres_tol = 1e-9;
  o->refine_maxit = 20;
  o->inner_tol = 1e-3;
  o->l_eps_mixed = 1e-3;
  o->precond = 0;
  o->gamma_re = 0.0;
  o->gamma_im_k = 1.0;
  o->far_direct = 0;
  o->interior = 0;
  o->translate_shape = 0;
  o->near_split = 0;
  o->far_rows = 0;
  o->use_graphs = 1;
}

// rule tables live in each device's constant memory: uploaded once per
// device; the flag and the upload are under one lock, so that threads setting
// up meshes at the same time neither upload twice nor read a half-set flag
void upload_rules() {
  static std::mutex mu;
  static bool done[64] = {};
  int dev = 0;
  BEM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error(BEM_E_HIP, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (done[dev]) return;
  double a[kRulePoints], b[kRulePoints], w[kRulePoints];
  int off[kMaxRuleOrder + 1];
  int pos = 0;
  for (int m = 1; m <= kMaxRuleOrder; ++m) {
    off[m - 1] = pos;
    std::vector<double> xi, wx, eta, we;
    gauss_jacobi_xi01(m, xi, wx);
    gauss_legendre01(m, eta, we);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        a[pos] = xi[i] * (1.0 - eta[j]);
        b[pos] = xi[i] * eta[j];
        w[pos] = wx[i] * we[j];
        ++pos;
      }
  }
  off[kMaxRuleOrder] = pos;
  upload_rule_tables(a, b, w, off);
  BEM_HIP(hipGetLastError());
  done[dev] = true;
}

int default_levels(int64_t N) {
  // 1 + round(log2(sqrt(N) / 22.5) / 2), at least 1
  double v = 0.5 * std::log2(std::sqrt(double(N)) / 22.5);
  return std::max(1, 1 + (int)std::floor(v + 0.5));
}

void check_options(const bem_options* o) {
  if (!o) throw Error(BEM_E_ARG, "options is NULL");
  if (o->quad_m_max < 1 || o->quad_m_max > kMaxRuleOrder) throw Error(BEM_E_ARG, "quad_m_max must be in [1, 8]");
  if (!(o->quad_eps > 0.0)) throw Error(BEM_E_ARG, "quad_eps must be positive");
  if (!(o->quad_eps_mixed > 0.0)) throw Error(BEM_E_ARG, "quad_eps_mixed must be positive");
  if (!(o->subdiv_ratio > 0.0)) throw Error(BEM_E_ARG, "subdiv_ratio must be positive");
  if (o->max_subdiv < 0 || o->max_subdiv > 15) throw Error(BEM_E_ARG, "max_subdiv must be in [0, 15]");
  if (o->self_n < 1 || o->self_n > 64) throw Error(BEM_E_ARG, "self_n must be in [1, 64]");
  if (o->edge_parts < 1 || o->edge_gauss < 1 || o->edge_parts * o->edge_gauss > 4096)
    throw Error(BEM_E_ARG, "invalid edge rule");
  if (o->gmres_restart < 1 || o->gmres_restart > 200) throw Error(BEM_E_ARG, "gmres_restart must be in [1, 200]");
  if (o->gmres_maxit < 1) throw Error(BEM_E_ARG, "gmres_maxit must be positive");
  if (!(o->gmres_tol > 0.0)) throw Error(BEM_E_ARG, "gmres_tol must be positive");
  if (o->use_fmm) {
    if (o->levels < 0 || o->levels > 16) throw Error(BEM_E_ARG, "levels must be in [0, 16]");
    if (o->leaf_size < 1) throw Error(BEM_E_ARG, "leaf_size must be positive");
    if (!(o->admissibility > 0.0)) throw Error(BEM_E_ARG, "admissibility must be positive");
    if (o->t_order < 1 || o->t_order > kMaxRuleOrder) throw Error(BEM_E_ARG, "t_order must be in [1, 8]");
  }
  if (o->precision != BEM_PREC_FP64 && o->precision != BEM_PREC_MIXED)
    throw Error(BEM_E_ARG, "unknown precision");
  if (o->precond < 0 || o->precond > 2) throw Error(BEM_E_ARG, "precond must be 0, 1 or 2");
  if (o->far_direct < 0 || o->far_direct > 2) throw Error(BEM_E_ARG, "far_direct must be 0, 1 or 2");
  if (o->interior != 0 && o->interior != 1) throw Error(BEM_E_ARG, "interior must be 0 or 1");
  {
    const int t = o->translate_shape & ~kTranslateFlags;
    if (o->translate_shape < 0 || (t != 0 && t != 64 && t != 128 && t != 256) ||
        (o->translate_shape & kTranslateFlags) == kTranslateFlags)
      throw Error(BEM_E_ARG, "translate_shape must be 0, 64, 128 or 256, plus 4096 for the slab order or 8192 "
                             "for the node-range order");
  }
  if (o->near_split < 0 || o->near_split > 100) throw Error(BEM_E_ARG, "near_split must be in [0, 100]");
  if (o->far_rows != 0 && o->far_rows != 1 && o->far_rows != kFarRows)
    throw Error(BEM_E_ARG, "far_rows must be 0, 1 or " + std::to_string(kFarRows));
  if (o->use_graphs != 0 && o->use_graphs != 1) throw Error(BEM_E_ARG, "use_graphs must be 0 or 1");
  if (o->level_rows != 0 && o->level_rows != 1) throw Error(BEM_E_ARG, "level_rows must be 0 or 1");
  if (o->solver != 0 && o->solver != 1) throw Error(BEM_E_ARG, "solver must be 0 (GMRES) or 1 (CGS)");
  if (o->near_waves_per_cu < 0 || o->near_waves_per_cu > 64)
    throw Error(BEM_E_ARG, "near_waves_per_cu must be in [0, 64]");
  if (o->far_direct && !o->use_fmm) throw Error(BEM_E_ARG, "far_direct needs the cluster tree (use_fmm = 1)");
  if (!std::isfinite(o->gamma_re) || !std::isfinite(o->gamma_im_k) || o->gamma_im_k == 0.0)
    throw Error(BEM_E_ARG, "the coupling needs a finite gamma with a non-zero imaginary part");
}

}  // namespace

namespace bem {

void set_last_error(const std::string& msg) { g_last_error = msg; }
void clear_last_error() { g_last_error.clear(); }

namespace {
std::mutex g_alloc_mu;
AllocHook g_alloc_hook;
}  // namespace

AllocHook current_alloc_hook() {
  std::lock_guard<std::mutex> lock(g_alloc_mu);
  return g_alloc_hook;
}

void apply_tree(bem_mesh* m, bem_op op, bem_precision prec, const double2* x, double2* y, hipStream_t s) {
  apply_tree_part(m, op, prec, 0, x, y, s);
}

void apply_tree_part_ext(bem_mesh* m, bem_op op, bem_precision prec, int part, const double2* x, double2* y,
                         hipStream_t s, bool vmode);

// The exterior application, turned into the interior one when the mesh was
// made for an interior problem.
void apply_one(bem_mesh* m, bem_op op, bem_precision prec, int part, const double2* x, double2* y,
               hipStream_t s, bool vmode) {
  apply_tree_part_ext(m, op, prec, part, x, y, s, vmode);
  if (!m->opt.interior) return;
  const bool adj = op != BEM_OP_A;
  const int mode = part == 2 ? 4 : (vmode ? 2 : 0) + (adj ? 1 : 0);
  launch_interior(m->N, mode, m->gre, m->gim, m->have_beta ? m->d_cfac.p : nullptr, x, y, s);
}

void apply_tree_part(bem_mesh* m, bem_op op, bem_precision prec, int part, const double2* x, double2* y,
                     hipStream_t s, bool vmode) {
  if (!m->has_pres || vmode) {
    apply_one(m, op, prec, part, x, y, s, vmode);
    return;
  }
  // PRES columns are those of V: M x = A (x off PRES) + V (x on PRES);
  // M^H y = A^H y off PRES, V^H y on PRES (rows of the transpose)
  if (op == BEM_OP_A) {
    launch_mask(m->N, m->d_pres.p, 0, x, m->d_px.p, s);
    apply_one(m, op, prec, part, m->d_px.p, y, s, false);
    launch_mask(m->N, m->d_pres.p, 1, x, m->d_px.p, s);
    apply_one(m, op, prec, part, m->d_px.p, m->d_py.p, s, true);
    launch_axpby(m->N, make_double2(1, 0), y, make_double2(1, 0), m->d_py.p, y, s);
  } else {
    apply_one(m, op, prec, part, x, y, s, false);
    apply_one(m, op, prec, part, x, m->d_py.p, s, true);
    launch_blend(m->N, m->d_pres.p, y, m->d_py.p, s);
  }
}

void apply_tree_part_ext(bem_mesh* m, bem_op op, bem_precision prec, int part, const double2* x, double2* y,
                         hipStream_t s, bool vmode) {
  // a caller's own graph capture of s also counts as capturing (the far field
  // then forks no third stream; see fmm_apply)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  BEM_HIP(hipStreamIsCapturing(s, &cs));
  struct CaptureFlag {
    bem_mesh* m;
    bool was;
    ~CaptureFlag() { m->capturing = was; }
  } flag{m, m->capturing};
  if (cs != hipStreamCaptureStatusNone) m->capturing = true;
  if (part == 2) {
    BEM_HIP(hipMemsetAsync(y, 0, m->N * sizeof(double2), s));
    far_apply(m, op, prec, x, y, s, vmode);
    return;
  }
  NearLaunch L{};
  L.N = m->N;
  L.Q = quad_recs(m);
  L.geom = m->d_geom.p;
  L.geom32 = m->d_geom32.p;
  L.cfac = m->have_beta ? m->d_cfac.p : nullptr;
  L.diag = m->d_diag.p;
  L.vdiag = m->d_vdiag.p;
  L.k = m->k;
  L.gre = m->gre;
  L.gim = m->gim;
  L.wpb = m->tune_wpb[prec == BEM_PREC_FP64 ? 0 : 1];
  L.order = m->d_order.p;
  L.rec = m->d_rec.p;
  L.rec32 = m->d_rec32.p;
  L.kap = m->kap;
  L.kap32 = m->kap32;
  // a resident near-field grid only while the far field runs beside it
  L.nwaves = part == 0 && m->fmm ? (int64_t)m->tune_nwaves[prec == BEM_PREC_FP64 ? 0 : 1] * m->n_cu : 0;
  if (op == BEM_OP_A) {
    L.off = m->d_off.p;
    L.seg = m->d_seg.p;
    L.items = m->d_items.p;
  } else {
    ensure_transposed_plan(m, s);
    L.off = m->d_off_t.p;
    L.seg = m->d_seg_t.p;
    L.items = m->d_items_t.p;
  }
  if (part == 0 && m->fmm) {
    // fork: far field into d_far on the side stream, near field into y on s
    // (stream, events and buffer are made with the mesh: nothing here may
    // allocate, so that the sequence can be captured).  The near field is
    // enqueued first: after an idle device (each Krylov step waits for its
    // Gram-Schmidt values) it would otherwise start only once the host has
    // submitted the whole far-field chain.
    BEM_HIP(hipEventRecord(m->ev_fork, s));
    BEM_HIP(hipStreamWaitEvent(m->side_stream, m->ev_fork, 0));
    // With a resident near-field grid the targets may be split: the first
    // share (in visiting order) runs beside the far field, the rest one
    // wavefront each on the far field's stream once it is done, at full
    // occupancy.  Every target keeps one owner: results are identical.
    const int split = m->tune_split[prec == BEM_PREC_FP64 ? 0 : 1];
    const bool halves = op == BEM_OP_A && !vmode && L.nwaves > 0 && split > 0 && split < 100 && m->N >= 2;
    NearLaunch L1 = L, L2 = L;
    if (halves) {
      L1.count = std::max<int64_t>(1, std::min<int64_t>(m->N - 1, m->N * split / 100));
      L2.first = L1.count;
      L2.count = m->N - L1.count;
      L2.nwaves = 0;
    }
    launch_near(L1, prec == BEM_PREC_FP64, op != BEM_OP_A, vmode, x, y, s);
    launch_zero(m->N, m->d_far.p, m->side_stream);
    far_apply(m, op, prec, x, m->d_far.p, m->side_stream, vmode);
    if (halves) launch_near(L2, prec == BEM_PREC_FP64, false, false, x, y, m->side_stream);
    BEM_HIP(hipEventRecord(m->ev_join, m->side_stream));
    BEM_HIP(hipStreamWaitEvent(s, m->ev_join, 0));
    launch_axpby(m->N, make_double2(1, 0), y, make_double2(1, 0), m->d_far.p, y, s);
    BEM_HIP(hipGetLastError());
    return;
  }
  launch_near(L, prec == BEM_PREC_FP64, op != BEM_OP_A, vmode, x, y, s);
  BEM_HIP(hipGetLastError());
}

void far_apply(bem_mesh* m, bem_op op, bem_precision prec, const double2* x, double2* y, hipStream_t s, bool vmode) {
  if (!m->fmm) return;
  if (!m->far_direct && !(m->far_direct64 && prec == BEM_PREC_FP64)) {
    fmm_apply(m, op, prec, x, y, s, vmode);
    return;
  }
  FarLaunch F{};
  F.N = m->N;
  F.Q = quad_recs(m);
  F.geom = m->d_geom.p;
  F.geom32 = m->d_geom32.p;
  F.cfac = m->have_beta ? m->d_cfac.p : nullptr;
  F.elem_leaf = m->d_elem_leaf.p;
  F.far_off = m->d_far_off.p;
  F.far_beg = m->d_far_beg.p;
  F.far_end = m->d_far_end.p;
  for (int q = 0; q < kMaxRuleOrder; ++q) {
    F.rt2_min[q] = m->far_rt2_min[q];
    F.rt2_min32[q] = m->far_rt2_min32[q];
  }
  F.ratio2 = m->opt.subdiv_ratio * m->opt.subdiv_ratio;
  F.m_max = m->opt.quad_m_max;
  F.split_on_cap = m->opt.quad_split_on_cap;
  F.max_subdiv = m->opt.max_subdiv;
  F.k = m->k;
  F.gre = m->gre;
  F.gim = m->gim;
  F.rec = m->d_rec.p;
  F.rec32 = m->d_rec32.p;
  F.kap = m->kap;
  F.kap32 = m->kap32;
  // several points per wavefront pay in FP64, where the one-point kernel is
  // bound by the L2 traffic of its loads (35.1 -> 30.9 ms on a 40500-element
  // sphere); the FP32 kernel is bound by VALU issue and loses occupancy to
  // the larger register set (11.1 -> 14.6 ms)
  const bool rows = m->far_rows == kFarRows || (m->far_rows == 0 && prec == BEM_PREC_FP64);
  if (rows && m->d_far_grp.n > 0) {
    F.grp = m->d_far_grp.p;
    F.ngrp = (int64_t)m->d_far_grp.n;
  }
  launch_far_direct(F, prec == BEM_PREC_FP64, op != BEM_OP_A, vmode, x, y, s);
  BEM_HIP(hipGetLastError());
}

// Per leaf cluster, the element intervals (tree order) outside its near
// clusters, and the r~^2 thresholds of the rule orders for the direct far
// field: order m suffices iff all three a-priori estimates of Sec. 3.1.4 are
// below eps, i.e. iff q = 1/(2 r~) < q_m with q_m the smallest of the three
// roots.
void build_far_direct(bem_mesh* m, hipStream_t s) {
  const Level& leaf = m->tree.lv.back();
  std::vector<int32_t> el(m->N, -1);
  std::vector<int64_t> off(leaf.nc + 1, 0), fb, fe;
  for (int64_t c = 0; c < leaf.nc; ++c) {
    for (int64_t e = leaf.ebeg[c]; e < leaf.eend[c]; ++e) el[e] = (int32_t)c;
    std::vector<std::pair<int64_t, int64_t>> near;
    near.emplace_back(leaf.ebeg[c], leaf.eend[c]);
    for (int64_t q = leaf.nr_off[c]; q < leaf.nr_off[c + 1]; ++q)
      near.emplace_back(leaf.ebeg[leaf.nr[q]], leaf.eend[leaf.nr[q]]);
    std::sort(near.begin(), near.end());
    int64_t pos = 0;
    for (const auto& r : near) {
      if (r.first > pos) {
        fb.push_back(pos);
        fe.push_back(r.first);
      }
      pos = std::max(pos, r.second);
    }
    if (pos < m->N) {
      fb.push_back(pos);
      fe.push_back(m->N);
    }
    off[c + 1] = (int64_t)fb.size();
  }
  for (int64_t e = 0; e < m->N; ++e)
    if (el[e] < 0) throw Error(BEM_E_MESH, "element outside every leaf cluster", m->tree.perm[e]);
  for (int set = 0; set < 2; ++set) {
    const double eps = set == 0 ? m->opt.quad_eps : m->opt.quad_eps_mixed;
    for (int mm = 1; mm <= kMaxRuleOrder; ++mm) {
      const double q1 = std::pow(eps / 32.0, 1.0 / (2 * mm + 1));
      const double q2 = std::pow(eps / (64.0 * (2 * mm + 1)), 1.0 / (2 * mm + 2));
      const double q3 = std::pow(eps / (128.0 * (mm + 1) * (2 * mm + 1)), 1.0 / (2 * mm + 3));
      const double qm = std::min(q1, std::min(q2, q3));
      const double rt = 1.0 / (2.0 * qm);
      (set == 0 ? m->far_rt2_min : m->far_rt2_min32)[mm - 1] = rt * rt;
    }
  }
  std::vector<int64_t> grp;
  for (int64_t c = 0; c < leaf.nc; ++c)
    for (int64_t e = leaf.ebeg[c]; e < leaf.eend[c]; e += kFarRows)
      grp.push_back(e * 8 + (std::min<int64_t>(kFarRows, leaf.eend[c] - e) - 1));
  if (!grp.empty()) m->d_far_grp.upload(grp, s);
  m->d_elem_leaf.upload(el, s);
  m->d_far_off.upload(off, s);
  if (fb.empty()) {
    fb.push_back(0);
    fe.push_back(0);
  }
  m->d_far_beg.upload(fb, s);
  m->d_far_end.upload(fe, s);
}

BlockArgs block_args(const bem_mesh* m) {
  BlockArgs B{};
  B.nblk = m->nblk;
  B.elem_blk = m->d_elem_blk.p;
  B.beg = m->d_blk_beg.p;
  B.n = m->d_blk_n.p;
  B.off = m->d_blk_off.p;
  B.items = m->d_blk_items.p;
  B.seg = m->d_blk_seg.p;
  return B;
}

void precondition(bem_mesh* m, bem_op op, const double2* x, double2* y, hipStream_t s) {
  if (m->precond_ready) {
    launch_block_apply(m->N, block_args(m), m->d_blk_inv.p, op == BEM_OP_AH, x, y, s);
  } else {
    BEM_HIP(hipMemcpyAsync(y, x, m->N * sizeof(double2), hipMemcpyDeviceToDevice, s));
  }
}

// Partition the elements (tree order) into the preconditioner's blocks: each
// leaf cluster (the whole mesh without FMM) split evenly into pieces of at
// most max_n (<= kMaxBlock) elements.
void build_blocks(bem_mesh* m, int max_n, hipStream_t s) {
  std::vector<std::pair<int64_t, int64_t>> ranges;
  if (m->fmm) {
    const Level& leaf = m->tree.lv.back();
    for (int64_t c = 0; c < leaf.nc; ++c) ranges.emplace_back(leaf.ebeg[c], leaf.eend[c]);
  } else {
    ranges.emplace_back(0, m->N);
  }
  std::vector<int64_t> beg, off;
  std::vector<int32_t> nn, eb(m->N, -1);
  int64_t total = 0;
  for (const auto& r : ranges) {
    const int64_t len = r.second - r.first;
    if (len <= 0) continue;
    const int64_t pieces = (len + max_n - 1) / max_n;
    for (int64_t q = 0; q < pieces; ++q) {
      const int64_t pb = r.first + len * q / pieces, pe = r.first + len * (q + 1) / pieces;
      for (int64_t e = pb; e < pe; ++e) eb[e] = (int32_t)beg.size();
      beg.push_back(pb);
      nn.push_back((int32_t)(pe - pb));
      off.push_back(total);
      total += (pe - pb) * (pe - pb);
    }
  }
  for (int64_t e = 0; e < m->N; ++e)
    if (eb[e] < 0) throw Error(BEM_E_MESH, "element outside every leaf cluster", m->tree.perm[e]);
  // per row, the near items whose source lies in the row's block (order and
  // rule segments as in the plan): the assembly integrates only these
  std::vector<uint64_t> bitems;
  std::vector<int64_t> bseg((size_t)m->N * (kMaxRuleOrder + 1));
  for (int64_t t = 0; t < m->N; ++t) {
    const int64_t b0 = beg[eb[t]], b1 = b0 + nn[eb[t]];
    const int64_t* sg = m->plan->seg.data() + t * (kMaxRuleOrder + 1);
    for (int mc = 0; mc < kMaxRuleOrder; ++mc) {
      bseg[t * (kMaxRuleOrder + 1) + mc] = (int64_t)bitems.size();
      for (int64_t it = sg[mc]; it < sg[mc + 1]; ++it) {
        const int64_t j = m->g.owner((int64_t)(m->plan->items[it] & ((uint64_t(1) << 26) - 1)));
        if (j >= b0 && j < b1) bitems.push_back(m->plan->items[it]);
      }
    }
    bseg[t * (kMaxRuleOrder + 1) + kMaxRuleOrder] = (int64_t)bitems.size();
  }
  if (bitems.empty()) bitems.push_back(0);
  m->nblk = (int64_t)beg.size();
  m->blk_entries = total;
  m->d_blk_items.upload(bitems, s);
  m->d_blk_seg.upload(bseg, s);
  m->d_elem_blk.upload(eb, s);
  m->d_blk_beg.upload(beg, s);
  m->d_blk_n.upload(nn, s);
  m->d_blk_off.upload(off, s);
  m->d_blk_sing.alloc(m->nblk);
  m->d_blk_a.alloc(total);
  m->d_blk_inv.alloc(total);
}

// assemble and invert the blocks for the current problem
void setup_preconditioner(bem_mesh* m, hipStream_t s) {
  m->precond_ready = false;
  if (!m->opt.precond || m->nblk == 0 || m->has_pres) return;
  NearLaunch L{};
  L.N = m->N;
  L.Q = quad_recs(m);
  L.geom = m->d_geom.p;
  L.cfac = m->have_beta ? m->d_cfac.p : nullptr;
  L.diag = m->d_diag.p;
  L.off = m->d_off.p;
  L.seg = m->d_seg.p;
  L.items = m->d_items.p;
  L.k = m->k;
  L.gre = m->gre;
  L.gim = m->gim;
  L.rec = m->d_rec.p;
  L.kap = m->kap;
  const BlockArgs B = block_args(m);
  launch_block_assemble(L, B, m->d_blk_a.p, s);
  launch_block_invert(B, m->d_blk_a.p, m->d_blk_inv.p, m->d_blk_sing.p, s);
  BEM_HIP(hipGetLastError());
  std::vector<int32_t> sing(m->nblk);
  BEM_HIP(hipMemcpyAsync(sing.data(), m->d_blk_sing.p, m->nblk * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  BEM_HIP(hipStreamSynchronize(s));
  m->singular_blocks = 0;
  for (int32_t v : sing) m->singular_blocks += v;
  m->precond_ready = true;
}

void ensure_transposed_plan(bem_mesh* m, hipStream_t s) {
  if (m->have_plan_t) return;
  const NearPlan& P = *m->plan;
  const int64_t N = m->N;
  NearPlan T;
  T.off.assign(N + 1, 0);
  // items by the element of their source record; a quadrilateral's items
  // carry the half (0, 1) in bit 63
  const uint64_t jmask = (uint64_t(1) << 26) - 1;
  const Geometry& g = m->g;
  for (uint64_t it : P.items) T.off[g.owner((int64_t)(it & jmask)) + 1]++;
  for (int64_t j = 0; j < N; ++j) T.off[j + 1] += T.off[j];
  T.items.resize(P.items.size());
  std::vector<int64_t> pos(T.off.begin(), T.off.end() - 1);
  for (int64_t t = 0; t < N; ++t)
    for (int64_t q = P.off[t]; q < P.off[t + 1]; ++q) {
      uint64_t it = P.items[q];
      const int64_t r = (int64_t)(it & jmask);
      const int64_t j = g.owner(r);
      const uint64_t half = r >= N ? (uint64_t)((r - N) & 1) << 63 : 0;
      T.items[pos[j]++] = (it & ~jmask) | (uint64_t)t | half;
    }
  // sort each source's list by rule order for uniform wavefront work
  for (int64_t j = 0; j < N; ++j)
    std::stable_sort(T.items.begin() + T.off[j], T.items.begin() + T.off[j + 1],
                     [](uint64_t a, uint64_t b) { return ((a >> 26) & 7) < ((b >> 26) & 7); });
  T.pairs = P.pairs;
  T.points = P.points;
  T.max_m = P.max_m;
  build_segments(T, N);
  m->plan_t = std::move(T);
  m->d_off_t.upload(m->plan_t.off, s);
  m->d_seg_t.upload(m->plan_t.seg, s);
  m->d_items_t.upload(m->plan_t.items, s);
  BEM_HIP(hipStreamSynchronize(s));
  m->have_plan_t = true;
}

}  // namespace bem

namespace {

// Geometry, cluster tree and near-field plan on the host (no device work).
// el: n_tri x 4 vertex indices (el[4 e + 3] < 0: triangle)
// Geometry and cluster tree (the tree-order geometry g; without use_fmm the
// caller order and no tree).
void build_host_tree(int64_t n_nodes, const double* xyz, int64_t n_tri, const int32_t* tri, const bem_options& o,
                     Tree& tree, Geometry& g, int64_t& bad_element) {
  std::vector<int64_t> ident(n_tri);
  for (int64_t i = 0; i < n_tri; ++i) ident[i] = i;
  Geometry gc;
  try {
    gc = build_geometry(xyz, n_nodes, tri, n_tri, ident);
  } catch (const Error& e) {
    bad_element = e.element;
    throw;
  }
  if (o.use_fmm) {
    int levels = o.levels > 0 ? o.levels : default_levels(n_tri);
    tree = build_tree(gc, levels, o.root_box_edge, o.leaf_size, o.admissibility);
    g = build_geometry(xyz, n_nodes, tri, n_tri, tree.perm);
  } else {
    tree.perm = ident;
    tree.inv = ident;
    g = std::move(gc);
  }
}

// The near-field quadrature plan of a tree (all pairs without use_fmm).
void build_host_plan(const Tree& tree, const Geometry& g, const bem_options& o, NearPlan& plan,
                     int64_t& bad_element) {
  const int64_t n_tri = g.N;
  std::vector<int64_t> src_off, src_beg, src_end, tgt_group(n_tri, 0);
  if (o.use_fmm) {
    const Level& leaf = tree.lv.back();
    src_off.assign(leaf.nc + 1, 0);
    for (int64_t c = 0; c < leaf.nc; ++c) {
      for (int64_t e = leaf.ebeg[c]; e < leaf.eend[c]; ++e) tgt_group[e] = c;
      for (int64_t q = leaf.nr_off[c]; q < leaf.nr_off[c + 1]; ++q) {
        int64_t nb = leaf.nr[q];
        src_beg.push_back(leaf.ebeg[nb]);
        src_end.push_back(leaf.eend[nb]);
      }
      src_off[c + 1] = (int64_t)src_beg.size();
    }
  } else {
    src_off = {0, 1};
    src_beg = {0};
    src_end = {n_tri};
  }
  QuadParams q{o.quad_eps, o.quad_m_max, o.quad_split_on_cap, o.subdiv_ratio, o.max_subdiv};
  try {
    plan = build_near_plan(g, q, src_off, src_beg, src_end, tgt_group);
  } catch (const Error& e) {
    bad_element = e.element >= 0 ? tree.perm[e.element] : -1;
    throw Error(e.code, "more than max_subdiv nested subdivisions for element " + std::to_string(bad_element),
                bad_element);
  }
}

void build_host(int64_t n_nodes, const double* xyz, int64_t n_tri, const int32_t* tri, const bem_options& o,
                Tree& tree, Geometry& g, NearPlan& plan, int64_t& bad_element) {
  build_host_tree(n_nodes, xyz, n_tri, tri, o, tree, g, bad_element);
  build_host_plan(tree, g, o, plan, bad_element);
}

void validate_mesh_args(int64_t n_nodes, const double* xyz, int64_t n_tri, const int32_t* tri) {
  if (!xyz || !tri || n_nodes < 3 || n_tri < 1) throw Error(BEM_E_ARG, "empty or NULL mesh");
  for (int64_t i = 0; i < 3 * n_nodes; ++i)
    if (!std::isfinite(xyz[i])) throw Error(BEM_E_ARG, "non-finite node coordinate");
}

// triangles (n x 3) as the n x 4 element array of build_host
std::vector<int32_t> as_elements(int64_t n_tri, const int32_t* tri) {
  std::vector<int32_t> el((size_t)4 * n_tri);
  for (int64_t e = 0; e < n_tri; ++e) {
    for (int c = 0; c < 3; ++c) el[4 * e + c] = tri[3 * e + c];
    el[4 * e + 3] = -1;
  }
  return el;
}

}  // namespace

struct bem_tree {
  int64_t N = 0;
  bool fmm = false;
  Tree tree;
  Geometry g;
  bem_options opt{};
  // the near plan is built on first use (bem_tree_plan_stats, or a mesh made
  // from the tree, which shares it): the tree alone serves
  // bem_tree_fmm_lengths and the level queries.  The lock lets threads make
  // meshes of one tree at the same time.
  mutable std::shared_ptr<NearPlan> plan;
  mutable std::mutex plan_mu;
  const NearPlan& ensure_plan() const {
    std::lock_guard<std::mutex> lock(plan_mu);
    if (!plan) {
      auto p = std::make_shared<NearPlan>();
      int64_t bad = -1;
      build_host_plan(tree, g, opt, *p, bad);
      plan = std::move(p);
    }
    return *plan;
  }
};

extern "C" {

const char* bem_last_error(void) { return g_last_error.c_str(); }

bem_status bem_set_allocator(bem_alloc_fn alloc_fn, bem_free_fn free_fn, void* ctx) {
  return guarded([&]() -> bem_status {
    if ((alloc_fn == nullptr) != (free_fn == nullptr))
      return fail(BEM_E_ARG, "set both allocator functions, or neither (hipMalloc / hipFree)");
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    g_alloc_hook = AllocHook{alloc_fn, free_fn, alloc_fn ? ctx : nullptr};
    return BEM_OK;
  });
}

bem_status bem_options_default(bem_options* o, const char* preset) {
  return guarded([&]() -> bem_status {
    if (!o || !preset) return fail(BEM_E_ARG, "NULL argument");
    std::string p(preset);
    set_paper(o);
    if (p == "paper") return BEM_OK;
    if (p == "tight" || p == "mixed") {
      o->leaf_size = 32;
      o->admissibility = 3.0;
      o->l_mode = 1;
      o->l_eps = 1e-7;
      o->t_order = 6;
      o->quad_eps = 1e-8;
      o->quad_split_on_cap = 1;
      o->self_n = 12;
      o->edge_parts = 8;
      o->edge_gauss = 6;
      o->gmres_tol = 1e-6;
      o->l_eps_mixed = 1e-4;
      // complex-FP32 direct far field: the FP64 operator's rules, so that the
      // two operators differ by rounding only and each refinement step gains
      // the full inner reduction (the estimates do not see k: looser rules
      // for the FP32 operator drifted from the FP64 one at large k h)
      o->quad_eps_mixed = 1e-8;
      // the other sign of the imaginary coupling: the discrete spectrum lies
      // in the right half-plane, where block Jacobi also pays off
      o->gamma_im_k = -1.0;
      o->precond = 1;
      if (p == "mixed") o->precision = BEM_PREC_MIXED;
      return BEM_OK;
    }
    return fail(BEM_E_ARG, "unknown preset '" + p + "'");
  });
}

namespace {
bem_status create_mesh(int64_t n_nodes, const double* xyz, int64_t n_tri, const int32_t* tri,
                       const bem_options* o, void* stream, bem_mesh** out, const bem_tree* src = nullptr);
}

bem_status bem_mesh_create(int64_t n_nodes, const double* xyz, int64_t n_tri, const int32_t* tri,
                           const bem_options* o, void* stream, bem_mesh** out) {
  return guarded([&]() -> bem_status {
    if (!out) return fail(BEM_E_ARG, "out is NULL");
    *out = nullptr;
    validate_mesh_args(n_nodes, xyz, n_tri, tri);
    const std::vector<int32_t> el = as_elements(n_tri, tri);
    return create_mesh(n_nodes, xyz, n_tri, el.data(), o, stream, out);
  });
}

bem_status bem_mesh_create_elements(int64_t n_nodes, const double* xyz, int64_t n_el, const int32_t* el,
                                    const bem_options* o, void* stream, bem_mesh** out) {
  return guarded([&]() -> bem_status {
    if (!out) return fail(BEM_E_ARG, "out is NULL");
    *out = nullptr;
    validate_mesh_args(n_nodes, xyz, n_el, el);
    return create_mesh(n_nodes, xyz, n_el, el, o, stream, out);
  });
}

namespace {
// el: n_tri x 4 (validated by the caller); runs inside the caller's guard
bem_status create_mesh(int64_t n_nodes, const double* xyz, int64_t n_tri, const int32_t* tri,
                       const bem_options* o, void* stream, bem_mesh** out, const bem_tree* src) {
  {
    check_options(o);
    auto m = std::make_unique<bem_mesh>();
    m->opt = *o;
    m->N = n_tri;
    m->tune_nwaves[0] = m->tune_nwaves[1] = o->near_waves_per_cu;
    {
      const int t = o->translate_shape & ~kTranslateFlags;
      m->tune_tpb[0] = m->tune_tpb[1] = (t == 0 ? 64 : t) | (o->translate_shape & kTranslateFlags);
      m->tune_split[0] = m->tune_split[1] = o->near_split == 0 ? 100 : o->near_split;
      m->far_rows = o->far_rows;
    }
    m->fmm = o->use_fmm != 0;
    m->far_direct = o->far_direct == 1;
    m->far_direct64 = o->far_direct == 2;
    if (src) {
      // the host tree's geometry, tree and near plan (built there once)
      src->ensure_plan();
      m->tree = src->tree;
      m->g = src->g;
      m->plan = src->plan;
    } else {
      m->plan = std::make_shared<NearPlan>();
      build_host(n_nodes, xyz, n_tri, tri, *o, m->tree, m->g, *m->plan, m->bad_element);
    }
    {
      int dev = 0, ncu = 0;
      BEM_HIP(hipGetDevice(&dev));
      BEM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
      if (ncu > 0) m->n_cu = ncu;
    }
    upload_rules();
    hipStream_t s = as_stream(stream);
    m->d_geom.upload(m->g.f, s);
    std::vector<float> g32(m->g.f.begin(), m->g.f.end());
    m->d_geom32.upload(g32, s);
    if (m->g.nq > 0) {
      m->d_qidx.upload(m->g.qidx, s);
      m->d_hown.upload(m->g.hown, s);
      m->d_hq.upload(m->g.hq, s);
      std::vector<float> hq32(m->g.hq.begin(), m->g.hq.end());
      m->d_hq32.upload(hq32, s);
    }
    // integration records: the elements, then the quadrilaterals' halves
    m->d_rec.alloc((size_t)(n_tri + 2 * m->g.nq) * 16);
    m->d_rec32.alloc((size_t)(n_tri + 2 * m->g.nq) * 16);
    m->d_perm.upload(m->tree.perm, s);
    m->d_off.upload(m->plan->off, s);
    m->d_seg.upload(m->plan->seg, s);
    m->d_items.upload(m->plan->items, s);
    {
      // forward near-field schedule: groups of targets by decreasing work, the
      // work of a target being its wavefront passes (64 items each) weighted
      // by the rule's points plus a per-item setup of about two points
      std::vector<double> work(n_tri, 0.0);
      for (int64_t t = 0; t < n_tri; ++t)
        for (int mm = 1; mm <= kMaxRuleOrder; ++mm) {
          const int64_t cnt = m->plan->seg[t * (kMaxRuleOrder + 1) + mm] - m->plan->seg[t * (kMaxRuleOrder + 1) + mm - 1];
          work[t] += (double)((cnt + 63) / 64) * (mm * mm + 2);
        }
      // whole leaf clusters move together (their targets share sources, so
      // tree order within a cluster keeps the source data in cache)
      std::vector<std::pair<int64_t, int64_t>> groups;
      if (m->fmm) {
        const Level& leaf = m->tree.lv.back();
        for (int64_t c = 0; c < leaf.nc; ++c) groups.emplace_back(leaf.ebeg[c], leaf.eend[c]);
      } else {
        for (int64_t t = 0; t < n_tri; t += 64) groups.emplace_back(t, std::min<int64_t>(n_tri, t + 64));
      }
      std::vector<double> gw(groups.size(), 0.0);
      for (size_t q = 0; q < groups.size(); ++q)
        for (int64_t t = groups[q].first; t < groups[q].second; ++t) gw[q] += work[t];
      std::vector<size_t> go(groups.size());
      for (size_t q = 0; q < go.size(); ++q) go[q] = q;
      std::stable_sort(go.begin(), go.end(), [&](size_t a, size_t b) { return gw[a] > gw[b]; });
      std::vector<int32_t> order;
      order.reserve(n_tri);
      for (size_t q : go)
        for (int64_t t = groups[q].first; t < groups[q].second; ++t) order.push_back((int32_t)t);
      if ((int64_t)order.size() != n_tri) throw std::runtime_error("internal: leaf clusters do not cover the mesh");
      m->d_order.upload(order, s);
    }
    std::vector<double> u, w;
    gauss_legendre01(o->self_n, u, w);
    m->d_duffy_u.upload(u, s);
    m->d_duffy_w.upload(w, s);
    std::vector<double> gt, gw, et, ew;
    gauss_legendre01(o->edge_gauss, gt, gw);
    for (int p = 0; p < o->edge_parts; ++p)
      for (int i = 0; i < o->edge_gauss; ++i) {
        et.push_back((p + gt[i]) / o->edge_parts);
        ew.push_back(gw[i] / o->edge_parts);
      }
    m->d_edge_t.upload(et, s);
    m->d_edge_w.upload(ew, s);
    m->d_x.alloc(n_tri);
    m->d_y.alloc(n_tri);
    m->d_b.alloc(n_tri);
    m->d_sol.alloc(n_tri);
    m->d_cfac.alloc(n_tri);
    m->d_diag.alloc(n_tri);
    m->d_vdiag.alloc(n_tri);
    // the block-Jacobi factors hold blocks of the exterior operator
    if (o->precond && !o->interior) build_blocks(m.get(), o->precond == 1 ? kMaxBlock : 1, s);
    if (m->fmm) {
      BEM_HIP(hipStreamCreateWithFlags(&m->side_stream, hipStreamNonBlocking));
      BEM_HIP(hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming));
      BEM_HIP(hipEventCreateWithFlags(&m->ev_join, hipEventDisableTiming));
      BEM_HIP(hipStreamCreateWithFlags(&m->leaf_stream, hipStreamNonBlocking));
      BEM_HIP(hipEventCreateWithFlags(&m->ev_leaf_fork, hipEventDisableTiming));
      BEM_HIP(hipEventCreateWithFlags(&m->ev_leaf_join, hipEventDisableTiming));
      m->d_far.alloc(n_tri);
    }
    if (m->far_direct || m->far_direct64) build_far_direct(m.get(), s);
    BEM_HIP(hipStreamSynchronize(s));
    *out = m.release();
    return BEM_OK;
  }
}
}  // namespace

int64_t bem_mesh_bad_element(const bem_mesh* m) { return m ? m->bad_element : -1; }

bem_status bem_set_problem(bem_mesh* m, double k, const bem_c128* beta, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m) return fail(BEM_E_ARG, "mesh is NULL");
    if (!(k > 0.0) || !std::isfinite(k)) return fail(BEM_E_ARG, "k must be positive and finite");
    hipStream_t s = as_stream(stream);
    m->k = k;
    ++m->problem_stamp;
    m->gre = m->opt.gamma_re;
    m->gim = m->opt.gamma_im_k / k;  // gamma = i / k for (0, 1) (Sec. 2.5)
    m->have_beta = beta != nullptr;
    if (beta) {
      m->d_beta.alloc(m->N);
      BEM_HIP(hipMemcpyAsync(m->d_beta.p, beta, m->N * sizeof(double2), hipMemcpyDeviceToDevice, s));
      // c = -tau i k beta: the velocity -tau Y p along the outward normal
      launch_cfac(m->N, m->d_perm.p, m->d_beta.p, m->opt.interior ? -k : k, m->d_cfac.p, s);
      // admittance is ignored on PRES elements (their pressure is given)
      if (m->has_pres) launch_mask(m->N, m->d_pres.p, 0, m->d_cfac.p, m->d_cfac.p, s);
    }
    SelfLaunch L{};
    L.N = m->N;
    L.Q = quad_recs(m);
    L.geom = m->d_geom.p;
    L.cfac = m->have_beta ? m->d_cfac.p : nullptr;
    L.duffy_u = m->d_duffy_u.p;
    L.duffy_w = m->d_duffy_w.p;
    L.self_n = m->opt.self_n;
    L.edge_t = m->d_edge_t.p;
    L.edge_w = m->d_edge_w.p;
    L.edge_pts = m->opt.edge_parts * m->opt.edge_gauss;
    L.vdiag = m->d_vdiag.p;
    L.k = k;
    L.gre = m->gre;
    L.gim = m->gim;
    launch_self_terms(L, m->d_diag.p, s);
    // quadrature records: phase unit k (FP64, radians), k / (2 pi) (FP32, revolutions)
    m->kap = k;
    m->kap32 = (double)(float)(k / (2.0 * M_PI));
    launch_records(m->N, m->d_geom.p, m->kap, m->kap32, m->d_rec.p, m->d_rec32.p, s);
    // the quadrilaterals' halves: records N .. N + 2 nq
    launch_records_at(2 * m->g.nq, m->d_hq.p, m->N, m->kap, m->kap32, m->d_rec.p, m->d_rec32.p, s);
    BEM_HIP(hipGetLastError());
    setup_preconditioner(m, s);
    if (m->fmm && !m->far_direct) fmm_setup_problem(m, s);
    m->have_problem = true;
    return BEM_OK;
  });
}

bem_status bem_rhs_plane_wave(bem_mesh* m, const double d[3], bem_c128 P0, bem_c128* rhs, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !d || !rhs) return fail(BEM_E_ARG, "NULL argument");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    double n = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (!(n > 0.0)) return fail(BEM_E_ARG, "direction must be non-zero");
    double du[3] = {d[0] / n, d[1] / n, d[2] / n};
    hipStream_t s = as_stream(stream);
    launch_rhs_plane(m->N, m->d_geom.p, m->k, m->gre, m->gim, du, P0.re, P0.im, m->d_y.p, s);
    launch_scatter(m->N, m->d_perm.p, m->d_y.p, reinterpret_cast<double2*>(rhs), s);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
  });
}

bem_status bem_rhs_point_source(bem_mesh* m, const double x0[3], bem_c128 P0, bem_c128* rhs, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !x0 || !rhs) return fail(BEM_E_ARG, "NULL argument");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    hipStream_t s = as_stream(stream);
    launch_rhs_point(m->N, m->d_geom.p, m->k, m->gre, m->gim, x0, P0.re, P0.im, m->d_y.p, s);
    launch_scatter(m->N, m->d_perm.p, m->d_y.p, reinterpret_cast<double2*>(rhs), s);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
  });
}

bem_status bem_incident_field(bem_mesh* m, int kind, const double src[3], bem_c128 P0, int64_t n_pts,
                              const double* pts, bem_c128* out, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !src || (n_pts > 0 && (!pts || !out)) || n_pts < 0) return fail(BEM_E_ARG, "NULL argument");
    if (kind != 0 && kind != 1) return fail(BEM_E_ARG, "kind must be 0 (plane wave) or 1 (point source)");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    double s3[3] = {src[0], src[1], src[2]};
    if (kind == 0) {
      const double n = std::sqrt(s3[0] * s3[0] + s3[1] * s3[1] + s3[2] * s3[2]);
      if (!(n > 0.0)) return fail(BEM_E_ARG, "direction must be non-zero");
      for (double& v : s3) v /= n;
    }
    hipStream_t s = as_stream(stream);
    launch_incident(n_pts, pts, kind, m->k, s3, P0.re, P0.im, reinterpret_cast<double2*>(out), s);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
  });
}

bem_status bem_autotune(bem_mesh* m, int32_t* near_wpb, int32_t* translate_tpb, int32_t* near_waves,
                        void* stream) {
  return guarded([&]() -> bem_status {
    if (!m) return fail(BEM_E_ARG, "mesh is NULL");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    hipStream_t s = as_stream(stream);
    hipEvent_t e0, e1;
    BEM_HIP(hipEventCreate(&e0));
    BEM_HIP(hipEventCreate(&e1));
    // the fastest of three batches of three runs after a warm-up: candidates
    // differ by a few per cent, about what one batch varies by
    auto timed = [&](auto&& fn) {
      fn();
      float best_ms = -1.0f;
      for (int batch = 0; batch < 3; ++batch) {
        BEM_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 3; ++r) fn();
        BEM_HIP(hipEventRecord(e1, s));
        BEM_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        BEM_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (best_ms < 0.0f || ms < best_ms) best_ms = ms;
      }
      return best_ms;
    };
    try {
      BEM_HIP(hipMemsetAsync(m->d_x.p, 0, m->N * sizeof(double2), s));
      for (int pi = 0; pi < 2; ++pi) {
        const bem_precision prec = pi == 0 ? BEM_PREC_FP64 : BEM_PREC_MIXED;
        float best = -1.0f;
        int pick = 4;
        for (int w : {1, 2, 4, 8}) {
          m->tune_wpb[pi] = w;
          const float t = timed([&] { apply_tree_part(m, BEM_OP_A, prec, 1, m->d_x.p, m->d_y.p, s); });
          if (best < 0.0f || t < best) {
            best = t;
            pick = w;
          }
        }
        m->tune_wpb[pi] = pick;
        if (m->fmm) {
          // resident near-field wavefronts per compute unit while the far
          // field runs beside it, jointly with the translation block size:
          // the kernels compete for the same slots, so both are timed on
          // whole applications
          best = -1.0f;
          int pick_nw = 0, pick_tpb = m->tune_tpb[pi], pick_late = 0;
          m->tune_split[pi] = 100;
          const bool direct = m->far_direct || (m->far_direct64 && pi == 0);
          const std::vector<int> tpbs = direct ? std::vector<int>{m->tune_tpb[pi]} : std::vector<int>{64, 128, 256};
          const std::vector<int> lates = direct ? std::vector<int>{0} : std::vector<int>{0, 1};
          for (int late : lates)
            for (int tpb : tpbs) {
              for (int nw : {0, 8, 12, 16, 24}) {
                m->tune_tpb[pi] = tpb;
                m->tune_nwaves[pi] = nw;
                m->tune_fork_late[pi] = late;
                const float t = timed([&] { apply_tree_part(m, BEM_OP_A, prec, 0, m->d_x.p, m->d_y.p, s); });
                if (best < 0.0f || t < best) {
                  best = t;
                  pick_nw = nw;
                  pick_tpb = tpb;
                  pick_late = late;
                }
              }
            }
          m->tune_nwaves[pi] = pick_nw;
          m->tune_tpb[pi] = pick_tpb;
          m->tune_fork_late[pi] = pick_late;
          if (!direct) {
            // the translation blocks in XCD slab order, then in XCD
            // node-range order, at each block size (a reordered grid can
            // prefer another size than the plain one), keeping the
            // near-field residency and fork point picked above
            int pick_shape = pick_tpb;
            for (int flag : {kTranslateSlab, kTranslateNodes})
              for (int tpb : tpbs) {
                m->tune_tpb[pi] = tpb | flag;
                const float t = timed([&] { apply_tree_part(m, BEM_OP_A, prec, 0, m->d_x.p, m->d_y.p, s); });
                if (t < best) {
                  best = t;
                  pick_shape = tpb | flag;
                }
              }
            m->tune_tpb[pi] = pick_shape;
          }
          // a resident near-field grid: the share of targets it keeps beside
          // the far field (the rest run after it at full occupancy)
          m->tune_split[pi] = 100;
          if (pick_nw > 0) {
            int pick_split = 100;
            for (int split : {90, 80, 70, 60, 50}) {
              m->tune_split[pi] = split;
              const float t = timed([&] { apply_tree_part(m, BEM_OP_A, prec, 0, m->d_x.p, m->d_y.p, s); });
              if (t < best) {
                best = t;
                pick_split = split;
              }
            }
            m->tune_split[pi] = pick_split;
          }
        }
        if (near_wpb) near_wpb[pi] = m->tune_wpb[pi];
        if (translate_tpb) translate_tpb[pi] = m->tune_tpb[pi];
        if (near_waves) near_waves[pi] = m->tune_nwaves[pi];
      }
      ++m->problem_stamp;  // captured applications used the old shapes
    } catch (...) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    BEM_HIP(hipEventDestroy(e0));
    BEM_HIP(hipEventDestroy(e1));
    return BEM_OK;
  });
}

bem_status bem_apply(bem_mesh* m, bem_op op, bem_precision prec, const bem_c128* x, bem_c128* y,
                     void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !x || !y) return fail(BEM_E_ARG, "NULL argument");
    if (op != BEM_OP_A && op != BEM_OP_AH) return fail(BEM_E_ARG, "unknown operator");
    if (prec != BEM_PREC_FP64 && prec != BEM_PREC_MIXED) return fail(BEM_E_ARG, "unknown precision");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    hipStream_t s = as_stream(stream);
    launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(x), m->d_x.p, s);
    apply_tree(m, op, prec, m->d_x.p, m->d_y.p, s);
    launch_scatter(m->N, m->d_perm.p, m->d_y.p, reinterpret_cast<double2*>(y), s);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
  });
}

bem_status bem_apply_part(bem_mesh* m, bem_op op, bem_precision prec, int part, const bem_c128* x,
                          bem_c128* y, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !x || !y) return fail(BEM_E_ARG, "NULL argument");
    if (op != BEM_OP_A && op != BEM_OP_AH) return fail(BEM_E_ARG, "unknown operator");
    if (prec != BEM_PREC_FP64 && prec != BEM_PREC_MIXED) return fail(BEM_E_ARG, "unknown precision");
    if (part < 0 || part > 2) return fail(BEM_E_ARG, "part must be 0, 1 or 2");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    hipStream_t s = as_stream(stream);
    launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(x), m->d_x.p, s);
    apply_tree_part(m, op, prec, part, m->d_x.p, m->d_y.p, s);
    launch_scatter(m->N, m->d_perm.p, m->d_y.p, reinterpret_cast<double2*>(y), s);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
  });
}

bem_status bem_apply_dc(bem_mesh* m, bem_op op, bem_precision prec, const bem_c128* x, bem_c128* y,
                        void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !x || !y) return fail(BEM_E_ARG, "NULL argument");
    if (op != BEM_OP_A && op != BEM_OP_AH) return fail(BEM_E_ARG, "unknown operator");
    if (prec != BEM_PREC_FP64 && prec != BEM_PREC_MIXED) return fail(BEM_E_ARG, "unknown precision");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    hipStream_t s = as_stream(stream);
    launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(x), m->d_x.p, s);
    apply_tree_part(m, op, prec, 0, m->d_x.p, m->d_y.p, s, true);
    launch_scatter(m->N, m->d_perm.p, m->d_y.p, reinterpret_cast<double2*>(y), s);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
  });
}

bem_status bem_set_pressure_elements(bem_mesh* m, int64_t n, const int64_t* elems, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || n < 0 || (n > 0 && !elems)) return fail(BEM_E_ARG, "NULL argument or negative count");
    std::vector<double> mask(m->N, 0.0);
    for (int64_t i = 0; i < n; ++i) {
      if (elems[i] < 0 || elems[i] >= m->N) return fail(BEM_E_ARG, "PRES element index out of range");
      mask[m->tree.inv[elems[i]]] = 1.0;
    }
    hipStream_t s = as_stream(stream);
    m->has_pres = n > 0;
    if (m->has_pres) {
      m->d_pres.upload(mask, s);
      m->d_px.alloc(m->N);
      m->d_py.alloc(m->N);
    }
    // the factors of the problem (c, diagonal, preconditioner, captured
    // graphs) depend on the PRES set: bem_set_problem must run again
    m->have_problem = false;
    m->precond_ready = false;
    ++m->problem_stamp;
    return BEM_OK;
  });
}

bem_status bem_rhs_pressure(bem_mesh* m, const bem_c128* pbar, bem_c128* rhs, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !pbar || !rhs) return fail(BEM_E_ARG, "NULL argument");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    if (!m->has_pres) return fail(BEM_E_STATE, "no PRES elements (bem_set_pressure_elements)");
    hipStream_t s = as_stream(stream);
    // d_b = A (pbar on PRES elements) in the caller's order; rhs -= d_b
    launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(pbar), m->d_y.p, s);
    launch_mask(m->N, m->d_pres.p, 1, m->d_y.p, m->d_x.p, s);
    apply_one(m, BEM_OP_A, BEM_PREC_FP64, 0, m->d_x.p, m->d_y.p, s, false);
    launch_scatter(m->N, m->d_perm.p, m->d_y.p, m->d_b.p, s);
    double2* r = reinterpret_cast<double2*>(rhs);
    launch_axpby(m->N, make_double2(1, 0), r, make_double2(-1, 0), m->d_b.p, r, s);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
  });
}

bem_status bem_rhs_velocity(bem_mesh* m, const bem_c128* u, double rho_c, bem_c128* rhs, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !u || !rhs) return fail(BEM_E_ARG, "NULL argument");
    if (!(rho_c > 0.0)) return fail(BEM_E_ARG, "rho_c must be positive");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    hipStream_t s = as_stream(stream);
    // d_b = V u in the caller's order, then rhs = rhs - i k rho_c d_b (d_b is
    // the solve's staging buffer, allocated with the mesh and free between calls)
    launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(u), m->d_x.p, s);
    apply_tree_part(m, BEM_OP_A, BEM_PREC_FP64, 0, m->d_x.p, m->d_y.p, s, true);
    launch_scatter(m->N, m->d_perm.p, m->d_y.p, m->d_b.p, s);
    double2* r = reinterpret_cast<double2*>(rhs);
    launch_axpby(m->N, make_double2(1, 0), r, make_double2(0, -m->k * rho_c), m->d_b.p, r, s);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
  });
}

}  // extern "C"

namespace bem {

QuadRecs quad_recs(const bem_mesh* m) {
  QuadRecs Q;
  if (m->g.nq > 0) {
    Q.nh = 2 * m->g.nq;
    Q.qidx = m->d_qidx.p;
    Q.hown = m->d_hown.p;
    Q.hq = m->d_hq.p;
    Q.hq32 = m->d_hq32.p;
  }
  return Q;
}

FieldArgs field_args(bem_mesh* m, int64_t npts, int part) {
  FieldArgs A{};
  A.N = m->N;
  A.Q = quad_recs(m);
  A.npts = npts;
  A.geom = m->d_geom.p;
  A.cfac = m->have_beta ? m->d_cfac.p : nullptr;
  A.k = m->k;
  A.eps = m->opt.quad_eps;
  A.ratio = m->opt.subdiv_ratio;
  A.m_max = m->opt.quad_m_max;
  A.split_on_cap = m->opt.quad_split_on_cap;
  A.max_subdiv = m->opt.max_subdiv;
  A.part = part;
  A.dpdn = nullptr;
  A.tau = m->opt.interior ? -1.0 : 1.0;
  return A;
}

void check_field_error(bem_mesh* m, const int64_t* err, hipStream_t s) {
  int64_t e = -1;
  BEM_HIP(hipMemcpyAsync(&e, err, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BEM_HIP(hipStreamSynchronize(s));
  if (e >= 0) {
    m->bad_element = m->tree.perm[e];
    throw Error(BEM_E_MESH, "field point too close to element " + std::to_string(m->bad_element) +
                                " (subdivision limit)", m->bad_element);
  }
}

}  // namespace bem

extern "C" {

bem_status bem_field(bem_mesh* m, int64_t n_pts, const double* pts, const bem_c128* p_surf,
                     const bem_c128* p_inc, bem_c128* p_out, double* energy, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !p_surf || n_pts < 0 || (n_pts > 0 && (!pts || !p_out))) return fail(BEM_E_ARG, "NULL argument");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    if (m->opt.interior)
      return fail(BEM_E_STATE, "field points use the exterior representation formula (interior mesh)");
    if (m->has_pres)
      return fail(BEM_E_STATE, "the mesh has PRES elements, whose normal derivative is not c p: use bem_field_pv");
    if (n_pts == 0) {
      if (energy) BEM_HIP(hipMemsetAsync(energy, 0, sizeof(double), as_stream(stream)));
      return BEM_OK;
    }
    hipStream_t s = as_stream(stream);
    DevBuf<int64_t> err;
    err.upload(std::vector<int64_t>{-1}, s);
    launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(p_surf), m->d_x.p, s);
    launch_field(field_args(m, n_pts, 0), pts, m->d_x.p, reinterpret_cast<const double2*>(p_inc),
                 reinterpret_cast<double2*>(p_out), err.p, s);
    if (energy) launch_energy(n_pts, reinterpret_cast<const double2*>(p_out), energy, s);
    BEM_HIP(hipGetLastError());
    check_field_error(m, err.p, s);
    return BEM_OK;
  });
}

bem_status bem_field_pv(bem_mesh* m, int64_t n_pts, const double* pts, const bem_c128* p_surf,
                        const bem_c128* dpdn_surf, const bem_c128* p_inc, bem_c128* p_out, double* energy,
                        void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !p_surf || !dpdn_surf || n_pts < 0 || (n_pts > 0 && (!pts || !p_out)))
      return fail(BEM_E_ARG, "NULL argument");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    hipStream_t s = as_stream(stream);
    if (n_pts == 0) {
      if (energy) BEM_HIP(hipMemsetAsync(energy, 0, sizeof(double), s));
      return BEM_OK;
    }
    DevBuf<int64_t> err;
    err.upload(std::vector<int64_t>{-1}, s);
    // both surface vectors into tree order (d_x: p, d_y: dp/dn; mesh staging)
    launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(p_surf), m->d_x.p, s);
    launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(dpdn_surf), m->d_y.p, s);
    FieldArgs A = field_args(m, n_pts, 0);
    A.dpdn = m->d_y.p;
    launch_field(A, pts, m->d_x.p, reinterpret_cast<const double2*>(p_inc), reinterpret_cast<double2*>(p_out),
                 err.p, s);
    if (energy) launch_energy(n_pts, reinterpret_cast<const double2*>(p_out), energy, s);
    BEM_HIP(hipGetLastError());
    check_field_error(m, err.p, s);
    return BEM_OK;
  });
}

bem_status bem_field_adjoint(bem_mesh* m, int64_t n_pts, const double* pts, const bem_c128* g, int part,
                             bem_c128* y_surf, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !y_surf || n_pts < 0 || (n_pts > 0 && (!pts || !g))) return fail(BEM_E_ARG, "NULL argument");
    if (part != 0 && part != 1) return fail(BEM_E_ARG, "part must be 0 or 1");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    if (m->opt.interior)
      return fail(BEM_E_STATE, "field points use the exterior representation formula (interior mesh)");
    if (m->has_pres) return fail(BEM_E_STATE, "the adjoint field map assumes dp/dn = c p (mesh has PRES elements)");
    hipStream_t s = as_stream(stream);
    DevBuf<int64_t> err;
    err.upload(std::vector<int64_t>{-1}, s);
    launch_field_adj(field_args(m, n_pts, part), pts, reinterpret_cast<const double2*>(g), m->d_y.p, err.p, s);
    launch_scatter(m->N, m->d_perm.p, m->d_y.p, reinterpret_cast<double2*>(y_surf), s);
    BEM_HIP(hipGetLastError());
    check_field_error(m, err.p, s);
    return BEM_OK;
  });
}

bem_status bem_grad_admittance(bem_mesh* m, const bem_c128* p, const bem_c128* w, const bem_c128* hg,
                               double rho_c, double* grad, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !p || !w || !hg || !grad) return fail(BEM_E_ARG, "NULL argument");
    if (!(rho_c > 0.0)) return fail(BEM_E_ARG, "rho_c must be positive");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    if (m->has_pres) return fail(BEM_E_STATE, "admittance gradients assume dp/dn = c p (mesh has PRES elements)");
    if (m->opt.interior) return fail(BEM_E_STATE, "admittance gradients are made for exterior problems");
    hipStream_t s = as_stream(stream);
    launch_grad_admittance(m->N, m->k, rho_c, reinterpret_cast<const double2*>(p),
                           reinterpret_cast<const double2*>(w), reinterpret_cast<const double2*>(hg), grad, s);
    BEM_HIP(hipGetLastError());
    return BEM_OK;
  });
}

bem_status bem_solve_adjoint(bem_mesh* m, const bem_c128* rhs, bem_c128* x_out, bem_solve_info* info,
                             void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !rhs || !x_out) return fail(BEM_E_ARG, "NULL argument");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    hipStream_t s = as_stream(stream);
    launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(rhs), m->d_b.p, s);
    SolveResult r = solve_tree(m, m->d_b.p, m->d_sol.p, s, BEM_OP_AH);
    launch_scatter(m->N, m->d_perm.p, m->d_sol.p, reinterpret_cast<double2*>(x_out), s);
    BEM_HIP(hipGetLastError());
    BEM_HIP(hipStreamSynchronize(s));
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->iterations = r.iterations;
      info->refinements = r.refinements;
      info->rel_residual = r.rel_residual;
      if (!r.converged) info->warnings |= BEM_WARN_NOT_CONVERGED;
    }
    if (!r.converged)
      return fail(BEM_E_NOCONV, "GMRES stopped at relative residual " + std::to_string(r.rel_residual));
    return BEM_OK;
  });
}

namespace {

// outputs of one solve: p (caller order) and the normal velocity
void solve_outputs(bem_mesh* m, bem_c128* p_out, bem_c128* v_out, double rho_c, hipStream_t s) {
  launch_scatter(m->N, m->d_perm.p, m->d_sol.p, reinterpret_cast<double2*>(p_out), s);
  if (v_out) {
    // v = -tau Y p = -tau beta p / rho_c
    launch_velocity(m->N, m->have_beta ? m->d_beta.p : nullptr, m->opt.interior ? -rho_c : rho_c,
                    reinterpret_cast<double2*>(p_out), reinterpret_cast<double2*>(v_out), s);
    if (m->has_pres)
      launch_velocity_pres(m->N, m->d_perm.p, m->d_pres.p, m->k, rho_c, reinterpret_cast<double2*>(p_out),
                           reinterpret_cast<double2*>(v_out), s);
  }
}

void fill_info(const bem_mesh* m, const SolveResult& r, bem_solve_info* info);

}  // namespace

bem_status bem_solve_batch(int32_t n, bem_mesh* const* meshes, const bem_c128* const* rhs, bem_c128* const* p_out,
                           bem_c128* const* v_out, double rho_c, bem_solve_info* infos, void* stream) {
  return guarded([&]() -> bem_status {
    if (n < 0 || (n > 0 && (!meshes || !rhs || !p_out))) return fail(BEM_E_ARG, "NULL argument");
    for (int32_t i = 0; i < n; ++i) {
      if (!meshes[i] || !rhs[i] || !p_out[i]) return fail(BEM_E_ARG, "NULL mesh or vector in the batch");
      if (!meshes[i]->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called on a mesh");
      for (int32_t q = 0; q < i; ++q)
        if (meshes[q] == meshes[i]) return fail(BEM_E_ARG, "a mesh appears twice in the batch");
      if (v_out && v_out[i] && !(rho_c > 0.0)) return fail(BEM_E_ARG, "rho_c must be positive when v_out is requested");
    }
    if (n == 0) return BEM_OK;
    hipStream_t s = as_stream(stream);
    // fork every system onto its mesh's stream after the caller's prior work
    std::vector<BatchItem> items;
    for (int32_t i = 0; i < n; ++i) {
      bem_mesh* m = meshes[i];
      if (!m->batch_stream) BEM_HIP(hipStreamCreateWithFlags(&m->batch_stream, hipStreamNonBlocking));
      if (!m->ev_batch) BEM_HIP(hipEventCreateWithFlags(&m->ev_batch, hipEventDisableTiming));
      BEM_HIP(hipEventRecord(m->ev_batch, s));
      BEM_HIP(hipStreamWaitEvent(m->batch_stream, m->ev_batch, 0));
      launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(rhs[i]), m->d_b.p, m->batch_stream);
      items.push_back(BatchItem{m, m->d_b.p, m->d_sol.p, m->batch_stream});
    }
    const std::vector<SolveResult> res = solve_tree_batch(items);
    bool all = true;
    for (int32_t i = 0; i < n; ++i) {
      bem_mesh* m = meshes[i];
      solve_outputs(m, p_out[i], v_out ? v_out[i] : nullptr, rho_c, m->batch_stream);
      BEM_HIP(hipEventRecord(m->ev_batch, m->batch_stream));
      BEM_HIP(hipStreamWaitEvent(s, m->ev_batch, 0));
      if (infos) fill_info(m, res[i], &infos[i]);
      all = all && res[i].converged;
    }
    BEM_HIP(hipGetLastError());
    BEM_HIP(hipStreamSynchronize(s));
    if (!all) return fail(BEM_E_NOCONV, "a system of the batch stopped before its tolerance");
    return BEM_OK;
  });
}

bem_status bem_solve(bem_mesh* m, const bem_c128* rhs, bem_c128* p_out, bem_c128* v_out, double rho_c,
                     bem_solve_info* info, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !rhs || !p_out) return fail(BEM_E_ARG, "NULL argument");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    if (v_out && !(rho_c > 0.0)) return fail(BEM_E_ARG, "rho_c must be positive when v_out is requested");
    hipStream_t s = as_stream(stream);
    launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(rhs), m->d_b.p, s);
    SolveResult r = solve_tree(m, m->d_b.p, m->d_sol.p, s);
    solve_outputs(m, p_out, v_out, rho_c, s);
    BEM_HIP(hipGetLastError());
    BEM_HIP(hipStreamSynchronize(s));
    if (info) fill_info(m, r, info);
    if (!r.converged)
      return fail(BEM_E_NOCONV, "GMRES stopped at relative residual " + std::to_string(r.rel_residual));
    return BEM_OK;
  });
}

namespace {

void fill_info(const bem_mesh* m, const SolveResult& r, bem_solve_info* info) {
  {
    {
      std::memset(info, 0, sizeof(*info));
      info->iterations = r.iterations;
      info->refinements = r.refinements;
      info->rel_residual = r.rel_residual;
      info->near_pairs = m->plan->pairs;
      info->near_items = (int64_t)m->plan->items.size();
      info->quad_points = m->plan->points;
      if (m->fmm) {
        info->levels = (int)m->tree.lv.size();
        for (int l = 0; l < info->levels && l < 16; ++l) {
          info->clusters[l] = (int32_t)m->tree.lv[l].nc;
          info->L[l] = m->fmm_L[l];
          info->L_mixed[l] = m->fmm_L32[l];
          if (m->fmm_L[l] > 30) info->warnings |= BEM_WARN_LARGE_L;
        }
      }
      if (!r.converged) info->warnings |= BEM_WARN_NOT_CONVERGED;
      // elements per wavelength from the mean element size sqrt(2 A) (equilateral edge ~ 1.52 sqrt(A))
      double asum = 0.0;
      for (int64_t e = 0; e < m->N; ++e) asum += m->g.at(G_AREA, e);
      double h = std::sqrt(4.0 / std::sqrt(3.0) * asum / double(m->N));
      double lambda = 2.0 * M_PI / m->k;
      if (lambda / h < 6.0) info->warnings |= BEM_WARN_COARSE_MESH;
    }
  }
}

}  // namespace

bem_status bem_mesh_launch_shapes(const bem_mesh* m, int32_t* near_wpb, int32_t* translate_shape,
                                  int32_t* near_waves, int32_t* near_split) {
  return guarded([&]() -> bem_status {
    if (!m) return fail(BEM_E_ARG, "mesh is NULL");
    for (int p = 0; p < 2; ++p) {
      if (near_wpb) near_wpb[p] = m->tune_wpb[p];
      if (translate_shape) translate_shape[p] = m->tune_tpb[p];
      if (near_waves) near_waves[p] = m->tune_nwaves[p];
      if (near_split) near_split[p] = m->tune_split[p];
    }
    return BEM_OK;
  });
}

bem_status bem_mesh_stats(const bem_mesh* m, int32_t* levels, int32_t* clusters, int64_t* near_pairs,
                          int64_t* near_items, int64_t* quad_points) {
  return guarded([&]() -> bem_status {
    if (!m) return fail(BEM_E_ARG, "mesh is NULL");
    int nl = m->fmm ? (int)m->tree.lv.size() : 0;
    if (levels) *levels = nl;
    if (clusters)
      for (int l = 0; l < nl; ++l) clusters[l] = (int32_t)m->tree.lv[l].nc;
    if (near_pairs) *near_pairs = m->plan->pairs;
    if (near_items) *near_items = (int64_t)m->plan->items.size();
    if (quad_points) *quad_points = m->plan->points;
    return BEM_OK;
  });
}

size_t bem_workspace_bytes(const bem_mesh* m) {
  if (!m) return 0;
  size_t b = m->d_geom.bytes() + m->d_geom32.bytes() + m->d_qidx.bytes() + m->d_hown.bytes() + m->d_hq.bytes() +
             m->d_hq32.bytes() + m->d_rec.bytes() + m->d_rec32.bytes() + m->d_perm.bytes() + m->d_off.bytes() + m->d_order.bytes() +
             m->d_items.bytes() + m->d_seg.bytes() + m->d_seg_t.bytes() + m->d_off_t.bytes() + m->d_items_t.bytes() + m->d_beta.bytes() +
             m->d_cfac.bytes() + m->d_diag.bytes() + m->d_vdiag.bytes() + m->d_x.bytes() + m->d_y.bytes() + m->d_r.bytes() +
             m->d_b.bytes() + m->d_sol.bytes() + m->d_tmp.bytes() + m->d_V.bytes() + m->d_w.bytes() +
             m->d_partial.bytes() + m->d_h.bytes() + m->d_z.bytes() + m->d_elem_blk.bytes() +
             m->d_blk_n.bytes() + m->d_blk_sing.bytes() + m->d_blk_beg.bytes() + m->d_blk_off.bytes() +
             m->d_blk_a.bytes() + m->d_blk_inv.bytes() + m->d_blk_items.bytes() + m->d_blk_seg.bytes() + m->d_far.bytes() +
             m->d_pres.bytes() + m->d_px.bytes() + m->d_py.bytes();
  return b + fmm_bytes(m);
}

bem_status bem_mesh_diameter(int64_t n_nodes, const double* xyz, double* diameter) {
  return guarded([&]() -> bem_status {
    if (!xyz || !diameter || n_nodes < 1) return fail(BEM_E_ARG, "NULL argument or no nodes");
    for (int64_t i = 0; i < 3 * n_nodes; ++i)
      if (!std::isfinite(xyz[i])) return fail(BEM_E_ARG, "non-finite node coordinate");
    // largest squared distance over all node pairs (each pair once)
    double best = 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(max : best)
    for (int64_t i = 0; i < n_nodes; ++i) {
      const double xi = xyz[3 * i], yi = xyz[3 * i + 1], zi = xyz[3 * i + 2];
      double b = 0.0;
      for (int64_t j = i + 1; j < n_nodes; ++j) {
        const double dx = xyz[3 * j] - xi, dy = xyz[3 * j + 1] - yi, dz = xyz[3 * j + 2] - zi;
        const double d2 = dx * dx + dy * dy + dz * dz;
        b = d2 > b ? d2 : b;
      }
      best = b > best ? b : best;
    }
    *diameter = std::sqrt(best);
    return BEM_OK;
  });
}

bem_status bem_auto_method(int32_t requested, int64_t n_tri, double diameter, double k, int32_t* method) {
  return guarded([&]() -> bem_status {
    if (!method) return fail(BEM_E_ARG, "method is NULL");
    if (requested != BEM_METHOD_BEM && requested != BEM_METHOD_SLFMM && requested != BEM_METHOD_MLFMM)
      return fail(BEM_E_ARG, "requested must be BEM_METHOD_BEM, BEM_METHOD_SLFMM or BEM_METHOD_MLFMM");
    if (n_tri < 1 || !(diameter > 0.0) || !std::isfinite(diameter) || !(k > 0.0) || !std::isfinite(k))
      return fail(BEM_E_ARG, "n_tri, diameter and k must be positive");
    int32_t m = requested;
    // more elements than the conventional method (20000) or the single-level
    // FMM (50000) is meant for: the faster method
    if (m == BEM_METHOD_BEM && n_tri > 20000) m = BEM_METHOD_SLFMM;
    if ((m == BEM_METHOD_BEM || m == BEM_METHOD_SLFMM) && n_tri > 50000) m = BEM_METHOD_MLFMM;
    // wavelengths the expansion cannot resolve: at 80 or more diameters no
    // FMM at all; longer than the diameter, one level only
    const double lambda = 2.0 * M_PI / k;
    if (m != BEM_METHOD_BEM && lambda >= 80.0 * diameter) m = BEM_METHOD_BEM;
    if (m == BEM_METHOD_MLFMM && lambda > diameter) m = BEM_METHOD_SLFMM;
    *method = m;
    return BEM_OK;
  });
}

bem_status bem_tree_build(int64_t n_nodes, const double* xyz, int64_t n_tri, const int32_t* tri,
                          const bem_options* o, bem_tree** out) {
  return guarded([&]() -> bem_status {
    if (!out) return fail(BEM_E_ARG, "out is NULL");
    *out = nullptr;
    validate_mesh_args(n_nodes, xyz, n_tri, tri);
    check_options(o);
    auto t = std::make_unique<bem_tree>();
    t->N = n_tri;
    t->fmm = o->use_fmm != 0;
    t->opt = *o;
    int64_t bad = -1;
    const std::vector<int32_t> el = as_elements(n_tri, tri);
    build_host_tree(n_nodes, xyz, n_tri, el.data(), *o, t->tree, t->g, bad);
    *out = t.release();
    return BEM_OK;
  });
}

bem_status bem_mesh_create_from_tree(const bem_tree* t, const bem_options* o, void* stream, bem_mesh** out) {
  return guarded([&]() -> bem_status {
    if (!out) return fail(BEM_E_ARG, "out is NULL");
    *out = nullptr;
    if (!t || !o) return fail(BEM_E_ARG, "NULL argument");
    const bem_options& a = t->opt;
    const bool same = a.use_fmm == o->use_fmm && a.levels == o->levels && a.leaf_size == o->leaf_size &&
                      a.root_box_edge == o->root_box_edge && a.admissibility == o->admissibility &&
                      a.quad_eps == o->quad_eps && a.quad_m_max == o->quad_m_max &&
                      a.quad_split_on_cap == o->quad_split_on_cap && a.subdiv_ratio == o->subdiv_ratio &&
                      a.max_subdiv == o->max_subdiv;
    if (!same)
      return fail(BEM_E_ARG, "the options' tree and near-plan fields (use_fmm, levels, leaf_size, root_box_edge, "
                             "admissibility, quad_eps, quad_m_max, quad_split_on_cap, subdiv_ratio, max_subdiv) "
                             "differ from the tree's");
    return create_mesh(0, nullptr, t->N, nullptr, o, stream, out, t);
  });
}

int32_t bem_tree_levels(const bem_tree* t) { return (t && t->fmm) ? (int32_t)t->tree.lv.size() : 0; }

bem_status bem_tree_level(const bem_tree* t, int32_t level, int64_t* nc, int64_t* n_il, int64_t* n_near) {
  return guarded([&]() -> bem_status {
    if (!t || level < 0 || level >= bem_tree_levels(t)) return fail(BEM_E_ARG, "invalid tree or level");
    const Level& L = t->tree.lv[level];
    if (nc) *nc = L.nc;
    if (n_il) *n_il = (int64_t)L.il.size();
    if (n_near) *n_near = (int64_t)L.nr.size();
    return BEM_OK;
  });
}

bem_status bem_tree_level_data(const bem_tree* t, int32_t level, double* z, double* r, int64_t* ebeg,
                               int64_t* eend, int64_t* parent, int64_t* il_off, int64_t* il, int64_t* near_off,
                               int64_t* near) {
  return guarded([&]() -> bem_status {
    if (!t || level < 0 || level >= bem_tree_levels(t)) return fail(BEM_E_ARG, "invalid tree or level");
    const Level& L = t->tree.lv[level];
    auto cp = [](auto* dst, const auto& v) {
      if (dst) std::copy(v.begin(), v.end(), dst);
    };
    cp(z, L.z);
    cp(r, L.r);
    cp(ebeg, L.ebeg);
    cp(eend, L.eend);
    cp(parent, L.parent);
    cp(il_off, L.il_off);
    cp(il, L.il);
    cp(near_off, L.nr_off);
    cp(near, L.nr);
    return BEM_OK;
  });
}

bem_status bem_tree_perm(const bem_tree* t, int64_t* perm) {
  return guarded([&]() -> bem_status {
    if (!t || !perm) return fail(BEM_E_ARG, "NULL argument");
    std::copy(t->tree.perm.begin(), t->tree.perm.end(), perm);
    return BEM_OK;
  });
}

bem_status bem_tree_plan_stats(const bem_tree* t, int64_t* pairs, int64_t* items, int64_t* points) {
  return guarded([&]() -> bem_status {
    if (!t) return fail(BEM_E_ARG, "NULL argument");
    const NearPlan& P = t->ensure_plan();
    if (pairs) *pairs = P.pairs;
    if (items) *items = (int64_t)P.items.size();
    if (points) *points = P.points;
    return BEM_OK;
  });
}

bem_status bem_tree_fmm_lengths(const bem_tree* t, double k, const bem_options* o, int32_t* L, int32_t* L32,
                                int32_t* capped, double* bytes) {
  return guarded([&]() -> bem_status {
    if (!t || !o) return fail(BEM_E_ARG, "NULL argument");
    if (!t->fmm) return fail(BEM_E_STATE, "the tree was built without use_fmm");
    if (!(k > 0.0) || !std::isfinite(k)) return fail(BEM_E_ARG, "k must be positive and finite");
    check_options(o);
    const FmmPlanInfo I = fmm_plan_info(t->tree, t->N, k, *o);
    for (int l = 0; l < I.levels && l < 16; ++l) {
      if (L) L[l] = I.L[l];
      if (L32) L32[l] = I.L32[l];
    }
    if (capped) *capped = (I.capped64 ? 1 : 0) | (I.capped32 ? 2 : 0);
    if (bytes) *bytes = I.bytes;
    return BEM_OK;
  });
}

void bem_tree_destroy(bem_tree* t) { delete t; }

void bem_mesh_destroy(bem_mesh* m) { delete m; }

}  // extern "C"
