// Host side of the FMM far field: per-frequency setup (truncation lengths,
// sphere grids, interpolation matrices, translation values, leaf
// aggregation / disaggregation rows) and the sequence of kernel launches of
// one application.
//
// Truncation length per level (Eq. (FMMTruncation) with r_max the largest
// cluster radius of the level, kd = 2 r_max k, rounded up):
//   L = max(l_min, ceil(kd + l_factor log10(kd + pi)));
// with l_mode = 1 additionally L >= ceil(kd + 1.8 digits^(2/3) kd^(1/3)) and
// L >= ceil(ln(eps)/ln(1/a)), digits = -log10(eps), a the admissibility, and
// L lowered (not below 4) while the rounding unit times (2L+1)|h_L(k X_min)|
// exceeds eps/10 (X_min the smallest centre distance of the level's
// interaction pairs): the growth of h_L at small arguments (Sec. 4.2) must
// not amplify rounding beyond the target.  The complex-FP32 operator of the
// mixed path uses its own lengths (eps = l_eps_mixed, FP32 rounding unit,
// cap applied in every mode).
//
// Sphere grid (Sec. 3.3.1): L Gauss-Legendre nodes in cos(theta) (ascending)
// times 2L azimuths phi_j = j pi / L, weights w_t pi / L (sum 4 pi), node
// index nu = t * 2L + j.
#include <algorithm>
#include <cmath>

#include "fmm.h"
#include "state.h"

namespace bem {

namespace {

struct FmmLevel {
  int L = 0, nu = 0;
  int64_t nc = 0;
  DevBuf<double> s, w, z;
  DevBuf<int64_t> il_off, il, pm, pn, code;
  int64_t npairs = 0;
  DevBuf<double2> D64;
  DevBuf<float2> D32;
  DevBuf<double2> sig64, loc64;
  DevBuf<float2> sig32, loc32;
  DevBuf<int64_t> cbeg, cend, parent;
  // element-to-cluster rows of this level (level_rows option): element ranges
  // of the clusters, element -> cluster map, T'/S' rows on this level's grid
  DevBuf<int64_t> ebeg, eend, ec;
  DevBuf<double2> T64, S64;
  DevBuf<float2> T32, S32;
  // transition from the children (next level) to this level's grid
  DevBuf<double2> shift64;
  DevBuf<float2> shift32;
  bool resample = false;
  int Lc = 0, nm = 0;
  DevBuf<double> Mi64, Ma64, MiT64, MaT64;   // MiT/MaT: transposed per order (adjoint)
  DevBuf<float> Mi32, Ma32, MiT32, MaT32;
  // twiddles exp(-+ i m phi_j): Ec/Ep/Ecc order-major for the inverse DFTs,
  // EcT/EpT/EpcT node-major for the forward DFTs (c: conjugated)
  DevBuf<double2> Ec64, Ep64, Ecc64, EcT64, EpT64, EpcT64, tA64, tB64;
  DevBuf<float2> Ec32, Ep32, Ecc32, EcT32, EpT32, EpcT32, tA32, tB32;
  // what depends only on the expansion lengths is kept across wavenumbers:
  // the sphere grid (L it was built for, theta nodes and weights on the
  // host) and the transfer tables (child and own L they were built for)
  int grid_L = -1;
  std::vector<double> xt_h, wt_h;
  int xfer_Lc = -1, xfer_Lp = -1;
  // tree-only: largest cluster radius, shortest interaction distance
  double rmax = 0.0, xmin = -1.0;
};

}  // namespace

// One parameter set of the far field: set 0 carries the FP64 operator, set 1
// the complex-FP32 operator of the mixed path (its own truncation lengths).
struct FmmSet {
  std::vector<FmmLevel> lv;
  int top = 0;  // first level with interaction pairs; levels above it carry nothing
  DevBuf<double2> T64, S64;
  DevBuf<float2> T32, S32;
};

struct FmmState {
  FmmSet set[2];
  DevBuf<int64_t> leaf_ebeg, leaf_eend, elem_cluster;
  DevBuf<double> ra, rb, rw;
  int nq = 0;
  int t_order = 0;
  double k_setup = -1.0;
  double gre_setup = 0.0, gim_setup = 0.0;
};

void fmm_destroy(FmmState* f) { delete f; }

namespace {

// |h_n(x)| of the spherical Hankel function by upward recurrence from
// h_0 = -i exp(ix)/x, h_1 = -exp(ix)(x + i)/x^2
double hankel_abs(int n, double x) {
  double h0r = std::sin(x) / x, h0i = -std::cos(x) / x;
  if (n == 0) return std::hypot(h0r, h0i);
  double h1r = (std::sin(x) - x * std::cos(x)) / (x * x), h1i = -(std::cos(x) + x * std::sin(x)) / (x * x);
  for (int l = 2; l <= n; ++l) {
    const double f = (2.0 * (l - 1) + 1.0) / x;
    const double hr = f * h1r - h0r, hi = f * h1i - h0i;
    h0r = h1r;
    h0i = h1i;
    h1r = hr;
    h1i = hi;
  }
  return std::hypot(h1r, h1i);
}

// x_min: smallest centre distance over the level's interaction pairs (< 0:
// none).  single: length of the complex-FP32 operator (accuracy l_eps_mixed,
// stability cap with FP32 rounding in every mode).
int truncation_length(double k, double rmax, const bem_options& o, double x_min, bool single) {
  const double kd = 2.0 * rmax * k;
  int L = std::max(o.l_min, (int)std::ceil(kd + o.l_factor * std::log10(kd + M_PI)));
  const double eps = single ? o.l_eps_mixed : o.l_eps;
  const double unit = single ? 1.1920928955078125e-07 : 2.220446049250313e-16;
  if (o.l_mode == 1) {
    const double digits = -std::log10(eps);
    L = std::max(L, (int)std::ceil(kd + 1.8 * std::pow(digits, 2.0 / 3.0) * std::pow(kd, 1.0 / 3.0)));
    L = std::max(L, (int)std::ceil(std::log(eps) / std::log(1.0 / o.admissibility)));
  }
  if (x_min >= 0.0 && (o.l_mode == 1 || single)) {
    // stability: rounding amplified by (2L+1)|h_L(k X_min)| must stay below eps/10
    const double x = k * x_min;
    while (L > 4 && unit * (2 * L + 1) * hankel_abs(L, x) > 0.1 * eps) --L;
  }
  return L;
}

void sphere_grid(int L, std::vector<double>& s, std::vector<double>& w, std::vector<double>& xt,
                 std::vector<double>& wt) {
  std::vector<double> x01, w01;
  gauss_legendre01(L, x01, w01);
  xt.resize(L);
  wt.resize(L);
  // exactly antipodal: node L-1-t is -node t, azimuth j+L is azimuth j + pi,
  // so that s(t, j) = -s(L-1-t, j+L) bit for bit
  for (int t = 0; t < L; ++t) {
    const int tm = L - 1 - t;
    if (t < tm) {
      xt[t] = 2.0 * x01[t] - 1.0;
      wt[t] = 2.0 * w01[t];
    } else if (t == tm) {
      xt[t] = 0.0;
      wt[t] = 2.0 * w01[t];
    } else {
      xt[t] = -xt[tm];
      wt[t] = wt[tm];
    }
  }
  s.resize(3 * 2 * L * L);
  w.resize(2 * L * L);
  for (int t = 0; t < L; ++t) {
    const double ct = xt[t], st = std::sqrt(1.0 - ct * ct);
    for (int j = 0; j < 2 * L; ++j) {
      const int v = t * 2 * L + j;
      const int jj = j < L ? j : j - L;
      const double ph = jj * M_PI / L;
      const double sg = j < L ? 1.0 : -1.0;
      s[3 * v] = sg * (st * std::cos(ph));
      s[3 * v + 1] = sg * (st * std::sin(ph));
      s[3 * v + 2] = ct;
      w[v] = wt[t] * M_PI / L;
    }
  }
}

// normalised associated Legendre Pbar_n^m(x), 0 <= m <= n < nmax, with
// int_{-1}^{1} Pbar^2 dx = 1/(2 pi); out[(m * nmax + n)]
void assoc_legendre(int nmax, double x, std::vector<double>& out) {
  out.assign((size_t)nmax * nmax, 0.0);
  const double sx = std::sqrt(std::max(0.0, 1.0 - x * x));
  double pmm = std::sqrt(1.0 / (4.0 * M_PI));
  for (int m = 0; m < nmax; ++m) {
    if (m > 0) pmm = -std::sqrt((2.0 * m + 1.0) / (2.0 * m)) * sx * pmm;
    out[(size_t)m * nmax + m] = pmm;
    if (m + 1 < nmax) {
      double p1 = std::sqrt(2.0 * m + 3.0) * x * pmm;
      out[(size_t)m * nmax + m + 1] = p1;
      double p0 = pmm;
      for (int n = m + 2; n < nmax; ++n) {
        const double a = std::sqrt((4.0 * n * n - 1.0) / (double(n) * n - double(m) * m));
        const double b = std::sqrt(((n - 1.0) * (n - 1.0) - double(m) * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
        const double p2 = a * (x * p1 - b * p0);
        out[(size_t)m * nmax + n] = p2;
        p0 = p1;
        p1 = p2;
      }
    }
  }
}

template <class T>
void upload_vec(DevBuf<T>& d, const std::vector<T>& h, hipStream_t s) { d.upload(h, s); }

void upload_tree(bem_mesh* m, FmmState* F, hipStream_t s) {
  const Tree& T = m->tree;
  const int nl = (int)T.lv.size();
  for (int si = 0; si < 2; ++si) F->set[si].lv.resize(nl);
  for (int si = 0; si < 2; ++si)
  for (int l = 0; l < nl; ++l) {
    const Level& L = T.lv[l];
    FmmLevel& D = F->set[si].lv[l];
    D.nc = L.nc;
    for (double r : L.r) D.rmax = std::max(D.rmax, r);
    for (int64_t c = 0; c < L.nc; ++c)
      for (int64_t q = L.il_off[c]; q < L.il_off[c + 1]; ++q) {
        const int64_t n = L.il[q];
        const double d0 = L.z[3 * c] - L.z[3 * n], d1 = L.z[3 * c + 1] - L.z[3 * n + 1],
                     d2 = L.z[3 * c + 2] - L.z[3 * n + 2];
        const double v = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        if (D.xmin < 0.0 || v < D.xmin) D.xmin = v;
      }
    upload_vec(D.z, L.z, s);
    upload_vec(D.il_off, L.il_off, s);
    upload_vec(D.il, L.il, s);
    std::vector<int64_t> pm, pn;
    for (int64_t c = 0; c < L.nc; ++c)
      for (int64_t q = L.il_off[c]; q < L.il_off[c + 1]; ++q) {
        pm.push_back(c);
        pn.push_back(L.il[q]);
      }
    // Translation values are stored once per unordered pair {m, n} (m < n),
    // for X = z_m - z_n: D(-X, s) = D(X, -s), and the sphere grid is exactly
    // symmetric under s -> -s, so pair (n, m) reads the same slot at the
    // antipodal node.  code[q] = 2 slot + (m > n) for interaction entry q = (m, n).
    // The lists are symmetric because the admissibility test is.
    std::vector<int64_t> upm, upn, code(pm.size());
    std::vector<int64_t> slot_of(pm.size(), -1);
    for (int64_t q = 0; q < (int64_t)pm.size(); ++q)
      if (pm[q] < pn[q]) {
        slot_of[q] = (int64_t)upm.size();
        upm.push_back(pm[q]);
        upn.push_back(pn[q]);
      }
    for (int64_t c = 0; c < L.nc; ++c)
      for (int64_t q = L.il_off[c]; q < L.il_off[c + 1]; ++q) {
        const int64_t n = L.il[q];
        if (c < n) {
          code[q] = 2 * slot_of[q];
          continue;
        }
        const int64_t* b = L.il.data() + L.il_off[n];
        const int64_t* e = L.il.data() + L.il_off[n + 1];
        const int64_t* f = std::lower_bound(b, e, c);
        if (f == e || *f != c || c == n) throw Error(BEM_E_STATE, "interaction lists are not symmetric");
        code[q] = 2 * slot_of[L.il_off[n] + (f - b)] + 1;
      }
    D.npairs = (int64_t)upm.size();
    upload_vec(D.pm, upm, s);
    upload_vec(D.pn, upn, s);
    upload_vec(D.code, code, s);
    upload_vec(D.parent, L.parent, s);
    if (l + 1 < nl) {
      upload_vec(D.cbeg, L.cbeg, s);
      upload_vec(D.cend, L.cend, s);
    }
    if (m->opt.level_rows) {
      upload_vec(D.ebeg, L.ebeg, s);
      upload_vec(D.eend, L.eend, s);
      std::vector<int64_t> lec(m->N, 0);
      for (int64_t c = 0; c < L.nc; ++c)
        for (int64_t e = L.ebeg[c]; e < L.eend[c]; ++e) lec[e] = c;
      upload_vec(D.ec, lec, s);
    }
  }
  const Level& leaf = T.lv.back();
  upload_vec(F->leaf_ebeg, leaf.ebeg, s);
  upload_vec(F->leaf_eend, leaf.eend, s);
  std::vector<int64_t> ec(m->N);
  for (int64_t c = 0; c < leaf.nc; ++c)
    for (int64_t e = leaf.ebeg[c]; e < leaf.eend[c]; ++e) ec[e] = c;
  upload_vec(F->elem_cluster, ec, s);
}

void upload_rule(FmmState* F, int order, hipStream_t s) {
  if (F->t_order == order) return;
  std::vector<double> xi, wx, eta, we, a, b, w;
  gauss_jacobi_xi01(order, xi, wx);
  gauss_legendre01(order, eta, we);
  for (int i = 0; i < order; ++i)
    for (int j = 0; j < order; ++j) {
      a.push_back(xi[i] * (1.0 - eta[j]));
      b.push_back(xi[i] * eta[j]);
      w.push_back(wx[i] * we[j]);
    }
  F->ra.upload(a, s);
  F->rb.upload(b, s);
  F->rw.upload(w, s);
  F->nq = order * order;
  F->t_order = order;
}

template <class V>
struct Pick;
template <>
struct Pick<double2> {
  static double2* sig(FmmLevel& l) { return l.sig64.p; }
  static double2* loc(FmmLevel& l) { return l.loc64.p; }
  static double2* D(FmmLevel& l) { return l.D64.p; }
  static double2* shift(FmmLevel& l) { return l.shift64.p; }
  static double2* Ec(FmmLevel& l) { return l.Ec64.p; }
  static double2* Ep(FmmLevel& l) { return l.Ep64.p; }
  static double2* tA(FmmLevel& l) { return l.tA64.p; }
  static double2* tB(FmmLevel& l) { return l.tB64.p; }
  static double* Mi(FmmLevel& l) { return l.Mi64.p; }
  static double* Ma(FmmLevel& l) { return l.Ma64.p; }
  static double* MiT(FmmLevel& l) { return l.MiT64.p; }
  static double* MaT(FmmLevel& l) { return l.MaT64.p; }
  static double2* Ecc(FmmLevel& l) { return l.Ecc64.p; }
  static double2* EcT(FmmLevel& l) { return l.EcT64.p; }
  static double2* EpT(FmmLevel& l) { return l.EpT64.p; }
  static double2* EpcT(FmmLevel& l) { return l.EpcT64.p; }
  static double2* T(FmmSet* f) { return f->T64.p; }
  static double2* S(FmmSet* f) { return f->S64.p; }
  static double2* Tl(FmmLevel& l) { return l.T64.p; }
  static double2* Sl(FmmLevel& l) { return l.S64.p; }
};
template <>
struct Pick<float2> {
  static float2* sig(FmmLevel& l) { return l.sig32.p; }
  static float2* loc(FmmLevel& l) { return l.loc32.p; }
  static float2* D(FmmLevel& l) { return l.D32.p; }
  static float2* shift(FmmLevel& l) { return l.shift32.p; }
  static float2* Ec(FmmLevel& l) { return l.Ec32.p; }
  static float2* Ep(FmmLevel& l) { return l.Ep32.p; }
  static float2* tA(FmmLevel& l) { return l.tA32.p; }
  static float2* tB(FmmLevel& l) { return l.tB32.p; }
  static float* Mi(FmmLevel& l) { return l.Mi32.p; }
  static float* Ma(FmmLevel& l) { return l.Ma32.p; }
  static float* MiT(FmmLevel& l) { return l.MiT32.p; }
  static float* MaT(FmmLevel& l) { return l.MaT32.p; }
  static float2* Ecc(FmmLevel& l) { return l.Ecc32.p; }
  static float2* EcT(FmmLevel& l) { return l.EcT32.p; }
  static float2* EpT(FmmLevel& l) { return l.EpT32.p; }
  static float2* EpcT(FmmLevel& l) { return l.EpcT32.p; }
  static float2* T(FmmSet* f) { return f->T32.p; }
  static float2* S(FmmSet* f) { return f->S32.p; }
  static float2* Tl(FmmLevel& l) { return l.T32.p; }
  static float2* Sl(FmmLevel& l) { return l.S32.p; }
};

FactorArgs factor_args(bem_mesh* m, const FmmLevel& leaf) {
  FactorArgs a{};
  a.N = m->N;
  a.s = leaf.s.p;
  a.n = m->d_geom.p + (int64_t)G_NX * m->N;
  a.cfac = m->have_beta ? m->d_cfac.p : nullptr;
  a.k = m->k;
  return a;
}

// vmode: apply dA/dc (plain aggregation rows) instead of A
template <typename T, typename V>
void fmm_apply_t(bem_mesh* m, FmmState* FS, const double2* x, double2* y, bool vmode, hipStream_t s) {
  using P = Pick<V>;
  FmmSet* F = &FS->set[sizeof(T) == sizeof(float) ? 1 : 0];
  const int nl = (int)F->lv.size();
  FmmLevel& leaf = F->lv[nl - 1];
  const FactorArgs fa = factor_args(m, leaf);
  if (m->opt.level_rows) {
    // every level straight from and to the elements: sig_l = T'_l x, loc_l = D_l sig_l, y += S'_l loc_l
    for (int l = F->top; l < nl; ++l) {
      FmmLevel& L = F->lv[l];
      if (L.npairs == 0) continue;
      const FactorArgs fl = factor_args(m, L);
      launch_fmm_aggregate<T, V>(L.nc, L.ebeg.p, L.eend.p, L.nu, P::Tl(L), vmode ? nullptr : &fl, x, P::sig(L), false,
                                 s);
      launch_fmm_translate<T, V>(L.nc, L.il_off.p, L.il.p, L.code.p, false, L.L, L.nu, P::D(L), P::sig(L), P::loc(L),
                                 m->tune_tpb[sizeof(T) == sizeof(float) ? 1 : 0], s);
      launch_fmm_disaggregate<T, V>(m->N, L.ec.p, L.nu, P::Sl(L), nullptr, P::loc(L), y, false, s);
    }
    BEM_HIP(hipGetLastError());
    return;
  }
  const int tpb = m->tune_tpb[sizeof(T) == sizeof(float) ? 1 : 0];
  launch_fmm_aggregate<T, V>(leaf.nc, FS->leaf_ebeg.p, FS->leaf_eend.p, leaf.nu, P::T(F), vmode ? nullptr : &fa, x,
                             P::sig(leaf), false, s);
  // The leaf translation needs only the leaf signatures and is the largest
  // far-field kernel: with a tree of more than one level it runs on its own
  // stream beside the upward pass, the upper translations and the downward
  // pass, which joins it before adding into the leaf local expansions.  Not
  // while s is being captured into a graph: a capture that forked a third
  // stream this way ended in a host crash inside the solve, cause not found,
  // so captured applications keep the single far-field stream.
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  BEM_HIP(hipStreamIsCapturing(s, &cap));
  const bool fork =
      F->top < nl - 1 && m->leaf_stream != nullptr && !m->capturing && cap == hipStreamCaptureStatusNone;
  // the fork comes right after aggregation, or (tune_fork_late) after the
  // leaf level's own transfer to the level above, whose many small blocks
  // otherwise wait for wavefront slots behind the translation's
  const bool late = fork && m->tune_fork_late[sizeof(T) == sizeof(float) ? 1 : 0] != 0;
  auto fork_leaf = [&]() {
    BEM_HIP(hipEventRecord(m->ev_leaf_fork, s));
    BEM_HIP(hipStreamWaitEvent(m->leaf_stream, m->ev_leaf_fork, 0));
    launch_fmm_translate<T, V>(leaf.nc, leaf.il_off.p, leaf.il.p, leaf.code.p, false, leaf.L, leaf.nu, P::D(leaf),
                               P::sig(leaf), P::loc(leaf), tpb, m->leaf_stream);
    BEM_HIP(hipEventRecord(m->ev_leaf_join, m->leaf_stream));
  };
  if (fork && !late) fork_leaf();
  for (int l = nl - 2; l >= F->top; --l) {
    FmmLevel& Lp = F->lv[l];
    FmmLevel& Lc = F->lv[l + 1];
    if (!Lp.resample) {
      launch_fmm_up_equal<T, V>(Lp.nc, Lp.cbeg.p, Lp.cend.p, Lp.nu, P::shift(Lp), P::sig(Lc), P::sig(Lp), s);
    } else {
      launch_fmm_dft<T, V>(Lc.nc, Lc.L, 2 * Lc.L, Lp.nm, P::sig(Lc), nullptr, nullptr, 0, P::EcT(Lp), P::tA(Lp), s);
      launch_fmm_theta<T, V>(Lc.nc, Lp.L, Lc.L, Lp.nm, Lc.L - 1, P::Mi(Lp), P::tA(Lp), P::tB(Lp), s);
      launch_fmm_up_idft<T, V>(Lp.nc, Lp.cbeg.p, Lp.cend.p, Lp.L, 2 * Lp.L, Lp.nm, P::tB(Lp), P::Ep(Lp),
                               P::shift(Lp), P::sig(Lp), s);
    }
    if (late && l == nl - 2) fork_leaf();
  }
  for (int l = F->top; l < (fork ? nl - 1 : nl); ++l) {
    FmmLevel& L = F->lv[l];
    launch_fmm_translate<T, V>(L.nc, L.il_off.p, L.il.p, L.code.p, false, L.L, L.nu, P::D(L), P::sig(L), P::loc(L),
                               tpb, s);
  }
  for (int l = F->top; l + 1 < nl; ++l) {
    FmmLevel& Lp = F->lv[l];
    FmmLevel& Lc = F->lv[l + 1];
    const bool into_leaf = fork && l + 2 == nl;
    if (!Lp.resample) {
      if (into_leaf) BEM_HIP(hipStreamWaitEvent(s, m->ev_leaf_join, 0));
      launch_fmm_down_equal<T, V>(Lc.nc, Lc.parent.p, Lp.nu, P::shift(Lp), P::loc(Lp), P::loc(Lc), s);
    } else {
      launch_fmm_dft<T, V>(Lc.nc, Lp.L, 2 * Lp.L, Lp.nm, P::loc(Lp), P::shift(Lp), Lc.parent.p, 1, P::EpT(Lp),
                           P::tA(Lp), s);
      launch_fmm_theta<T, V>(Lc.nc, Lc.L, Lp.L, Lp.nm, Lc.L - 1, P::Ma(Lp), P::tA(Lp), P::tB(Lp), s);
      if (into_leaf) BEM_HIP(hipStreamWaitEvent(s, m->ev_leaf_join, 0));
      launch_fmm_down_idft<T, V>(Lc.nc, Lc.L, 2 * Lc.L, Lp.nm, P::tB(Lp), P::Ec(Lp), P::loc(Lc), s);
    }
  }
  launch_fmm_disaggregate<T, V>(m->N, FS->elem_cluster.p, leaf.nu, P::S(F), nullptr, P::loc(leaf), y, false, s);
  BEM_HIP(hipGetLastError());
}

// Conjugate transpose of the far field: the forward steps in reverse order,
// each replaced by its conjugate transpose.  Adjoint variables reuse the
// loc (of the disaggregation side) and sig (of the aggregation side) buffers:
//   loc'_leaf = S'^H y;  loc'_p = sum_c shift_c * Anterp^H(loc'_c)   (leaf -> root)
//   sig'_l = D_l^H loc'_l;  sig'_c += Interp^H(conj(shift_c) * sig'_p) (root -> leaf)
//   y += T'^H sig'_leaf
template <typename T, typename V>
void fmm_apply_adj_t(bem_mesh* m, FmmState* FS, const double2* x, double2* y, bool vmode, hipStream_t s) {
  using P = Pick<V>;
  FmmSet* F = &FS->set[sizeof(T) == sizeof(float) ? 1 : 0];
  const int nl = (int)F->lv.size();
  FmmLevel& leaf = F->lv[nl - 1];
  if (m->opt.level_rows) {
    // conjugate transpose of each level: loc'_l = S'_l^H x, sig'_l = D_l^H loc'_l, y += T'_l^H sig'_l
    for (int l = F->top; l < nl; ++l) {
      FmmLevel& L = F->lv[l];
      if (L.npairs == 0) continue;
      const FactorArgs fl = factor_args(m, L);
      launch_fmm_aggregate<T, V>(L.nc, L.ebeg.p, L.eend.p, L.nu, P::Sl(L), nullptr, x, P::loc(L), true, s);
      launch_fmm_translate<T, V>(L.nc, L.il_off.p, L.il.p, L.code.p, true, L.L, L.nu, P::D(L), P::loc(L), P::sig(L),
                                 m->tune_tpb[sizeof(T) == sizeof(float) ? 1 : 0], s);
      launch_fmm_disaggregate<T, V>(m->N, L.ec.p, L.nu, P::Tl(L), vmode ? nullptr : &fl, P::sig(L), y, true, s);
    }
    BEM_HIP(hipGetLastError());
    return;
  }
  const FactorArgs fa = factor_args(m, leaf);
  launch_fmm_aggregate<T, V>(leaf.nc, FS->leaf_ebeg.p, FS->leaf_eend.p, leaf.nu, P::S(F), nullptr, x, P::loc(leaf),
                             true, s);
  for (int l = nl - 2; l >= F->top; --l) {
    FmmLevel& Lp = F->lv[l];
    FmmLevel& Lc = F->lv[l + 1];
    if (!Lp.resample) {
      launch_fmm_up_equal<T, V>(Lp.nc, Lp.cbeg.p, Lp.cend.p, Lp.nu, P::shift(Lp), P::loc(Lc), P::loc(Lp), s);
    } else {
      launch_fmm_dft<T, V>(Lc.nc, Lc.L, 2 * Lc.L, Lp.nm, P::loc(Lc), nullptr, nullptr, 0, P::EcT(Lp), P::tA(Lp), s);
      launch_fmm_theta<T, V>(Lc.nc, Lp.L, Lc.L, Lp.nm, Lc.L - 1, P::MaT(Lp), P::tA(Lp), P::tB(Lp), s);
      launch_fmm_up_idft<T, V>(Lp.nc, Lp.cbeg.p, Lp.cend.p, Lp.L, 2 * Lp.L, Lp.nm, P::tB(Lp), P::Ep(Lp),
                               P::shift(Lp), P::loc(Lp), s);
    }
  }
  for (int l = F->top; l < nl; ++l) {
    FmmLevel& L = F->lv[l];
    launch_fmm_translate<T, V>(L.nc, L.il_off.p, L.il.p, L.code.p, true, L.L, L.nu, P::D(L), P::loc(L), P::sig(L),
                               m->tune_tpb[sizeof(T) == sizeof(float) ? 1 : 0], s);
  }
  for (int l = F->top; l + 1 < nl; ++l) {
    FmmLevel& Lp = F->lv[l];
    FmmLevel& Lc = F->lv[l + 1];
    if (!Lp.resample) {
      launch_fmm_down_equal<T, V>(Lc.nc, Lc.parent.p, Lp.nu, P::shift(Lp), P::sig(Lp), P::sig(Lc), s);
    } else {
      launch_fmm_dft<T, V>(Lc.nc, Lp.L, 2 * Lp.L, Lp.nm, P::sig(Lp), P::shift(Lp), Lc.parent.p, 1, P::EpcT(Lp),
                           P::tA(Lp), s);
      launch_fmm_theta<T, V>(Lc.nc, Lc.L, Lp.L, Lp.nm, Lc.L - 1, P::MiT(Lp), P::tA(Lp), P::tB(Lp), s);
      launch_fmm_down_idft<T, V>(Lc.nc, Lc.L, 2 * Lc.L, Lp.nm, P::tB(Lp), P::Ecc(Lp), P::sig(Lc), s);
    }
  }
  launch_fmm_disaggregate<T, V>(m->N, FS->elem_cluster.p, leaf.nu, P::T(F), vmode ? nullptr : &fa, P::sig(leaf),
                                y, true, s);
  BEM_HIP(hipGetLastError());
}

}  // namespace

namespace {

void setup_set(bem_mesh* m, FmmState* FS, int si, hipStream_t s) {
  const bool single = si == 1;
  FmmSet* F = &FS->set[si];
  const bem_options& o = m->opt;
  const Tree& T = m->tree;
  const int nl = (int)T.lv.size();
  const double k = m->k;
  F->top = nl - 1;
  for (int l = 0; l < nl; ++l)
    if (F->lv[l].npairs > 0) {
      F->top = l;
      break;
    }
  for (int l = 0; l < F->top; ++l) {
    F->lv[l].L = 0;
    F->lv[l].nu = 0;
    if (single) m->fmm_L32[l] = 0;
    else m->fmm_L[l] = 0;
  }
  // (uploads are synchronous: DevBuf::upload waits for its copy)
  for (int l = F->top; l < nl; ++l) {
    FmmLevel& D = F->lv[l];
    D.L = truncation_length(k, D.rmax, o, D.xmin, single);
    if (D.L > 120) throw Error(BEM_E_ARG, "expansion length " + std::to_string(D.L) + " above the supported 120");
    if (single) m->fmm_L32[l] = D.L;
    else m->fmm_L[l] = D.L;
    D.nu = 2 * D.L * D.L;
    if (D.grid_L != D.L) {
      std::vector<double> sh, wh;
      sphere_grid(D.L, sh, wh, D.xt_h, D.wt_h);
      D.s.upload(sh, s);
      D.w.upload(wh, s);
      D.grid_L = D.L;
    }
    const size_t nd = (size_t)std::max<int64_t>(1, D.npairs) * D.nu;
    if (single) {
      D.D32.alloc(nd);
      D.sig32.alloc(D.nc * D.nu);
      D.loc32.alloc(D.nc * D.nu);
    } else {
      D.D64.alloc(nd);
      D.sig64.alloc(D.nc * D.nu);
      D.loc64.alloc(D.nc * D.nu);
    }
    launch_fmm_translation(D.npairs, D.pm.p, D.pn.p, D.z.p, D.s.p, D.nu, D.L, k, single ? nullptr : D.D64.p,
                           single ? D.D32.p : nullptr, s);
  }
  for (int l = F->top; l + 1 < nl && !o.level_rows; ++l) {
    FmmLevel& P = F->lv[l];
    FmmLevel& C = F->lv[l + 1];
    if (single) P.shift32.alloc(C.nc * P.nu);
    else P.shift64.alloc(C.nc * P.nu);
    launch_fmm_shift(C.nc, C.parent.p, P.z.p, C.z.p, P.s.p, P.nu, k, single ? nullptr : P.shift64.p,
                     single ? P.shift32.p : nullptr, s);
    P.resample = C.L != P.L;
    P.Lc = C.L;
    if (!P.resample) continue;
    const int Lc = C.L, Lp = P.L;
    const int nm = 2 * Lc - 1;
    P.nm = nm;
    const size_t tmp = (size_t)C.nc * std::max(Lc, Lp) * nm;
    if (single) {
      P.tA32.alloc(tmp);
      P.tB32.alloc(tmp);
    } else {
      P.tA64.alloc(tmp);
      P.tB64.alloc(tmp);
    }
    if (P.xfer_Lc == Lc && P.xfer_Lp == Lp) continue;  // tables of these lengths are in place
    P.xfer_Lc = Lc;
    P.xfer_Lp = Lp;
    const std::vector<double>& xtp = P.xt_h;
    const std::vector<double>& xtc = C.xt_h;
    const std::vector<double>& wtp = P.wt_h;
    const std::vector<double>& wtc = C.wt_h;
    // M'_m[tp][tc] = sum_{n=m}^{Lc-1} Pbar_n^m(x_tp) Pbar_n^m(x_tc)
    std::vector<std::vector<double>> Pp(Lp), Pc(Lc);
    for (int t = 0; t < Lp; ++t) assoc_legendre(Lc, xtp[t], Pp[t]);
    for (int t = 0; t < Lc; ++t) assoc_legendre(Lc, xtc[t], Pc[t]);
    // theta matrices stored [row out][row in][|m|]:
    //   Mi [tp][tc][m] = (pi/Lc) M'_m[tp][tc] w_tc   (interpolation, child -> parent)
    //   Ma [tc][tp][m] = (pi/Lp) M'_m[tp][tc] w_tp   (anterpolation, parent -> child)
    //   MaT[tp][tc][m] = Ma[tc][tp][m]               (conjugate transpose of anterpolation)
    //   MiT[tc][tp][m] = Mi[tp][tc][m]               (conjugate transpose of interpolation)
    std::vector<double> Mi((size_t)Lp * Lc * Lc), Ma((size_t)Lc * Lp * Lc), MiT(Ma.size()), MaT(Mi.size());
    for (int mm = 0; mm < Lc; ++mm)
      for (int tp = 0; tp < Lp; ++tp)
        for (int tc = 0; tc < Lc; ++tc) {
          double acc = 0.0;
          for (int n = mm; n < Lc; ++n) acc += Pp[tp][(size_t)mm * Lc + n] * Pc[tc][(size_t)mm * Lc + n];
          const double vi = (M_PI / Lc) * acc * wtc[tc];
          const double va = (M_PI / Lp) * acc * wtp[tp];
          Mi[((size_t)tp * Lc + tc) * Lc + mm] = vi;
          MaT[((size_t)tp * Lc + tc) * Lc + mm] = va;
          Ma[((size_t)tc * Lp + tp) * Lc + mm] = va;
          MiT[((size_t)tc * Lp + tp) * Lc + mm] = vi;
        }
    std::vector<double2> Ec((size_t)nm * 2 * Lc), Ep((size_t)nm * 2 * Lp);
    for (int mi = 0; mi < nm; ++mi) {
      const int mv = mi - (Lc - 1);
      for (int j = 0; j < 2 * Lc; ++j) {
        const double ph = -mv * (j * M_PI / Lc);
        Ec[(size_t)mi * 2 * Lc + j] = make_double2(std::cos(ph), std::sin(ph));
      }
      for (int j = 0; j < 2 * Lp; ++j) {
        const double ph = mv * (j * M_PI / Lp);
        Ep[(size_t)mi * 2 * Lp + j] = make_double2(std::cos(ph), std::sin(ph));
      }
    }
    std::vector<double2> Ecc(Ec.size()), EcT(Ec.size()), EpT(Ep.size()), EpcT(Ep.size());
    for (size_t i = 0; i < Ec.size(); ++i) Ecc[i] = make_double2(Ec[i].x, -Ec[i].y);
    for (int mi = 0; mi < nm; ++mi) {
      for (int j = 0; j < 2 * Lc; ++j) EcT[(size_t)j * nm + mi] = Ec[(size_t)mi * 2 * Lc + j];
      for (int j = 0; j < 2 * Lp; ++j) {
        const double2 e = Ep[(size_t)mi * 2 * Lp + j];
        EpT[(size_t)j * nm + mi] = e;
        EpcT[(size_t)j * nm + mi] = make_double2(e.x, -e.y);
      }
    }
    auto f32 = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };
    auto c32 = [](const std::vector<double2>& v) {
      std::vector<float2> o(v.size());
      for (size_t i = 0; i < v.size(); ++i) o[i] = make_float2((float)v[i].x, (float)v[i].y);
      return o;
    };
    if (single) {
      P.Mi32.upload(f32(Mi), s);
      P.Ma32.upload(f32(Ma), s);
      P.MiT32.upload(f32(MiT), s);
      P.MaT32.upload(f32(MaT), s);
      P.Ec32.upload(c32(Ec), s);
      P.Ep32.upload(c32(Ep), s);
      P.Ecc32.upload(c32(Ecc), s);
      P.EcT32.upload(c32(EcT), s);
      P.EpT32.upload(c32(EpT), s);
      P.EpcT32.upload(c32(EpcT), s);
    } else {
      P.Mi64.upload(Mi, s);
      P.Ma64.upload(Ma, s);
      P.MiT64.upload(MiT, s);
      P.MaT64.upload(MaT, s);
      P.Ec64.upload(Ec, s);
      P.Ep64.upload(Ep, s);
      P.Ecc64.upload(Ecc, s);
      P.EcT64.upload(EcT, s);
      P.EpT64.upload(EpT, s);
      P.EpcT64.upload(EpcT, s);
    }
  }
  if (o.level_rows) {
    // the paper's explicit element-to-cluster rows on every level with pairs
    for (int l = F->top; l < nl; ++l) {
      FmmLevel& L = F->lv[l];
      if (L.npairs == 0) continue;
      if (single) {
        L.T32.alloc(m->N * L.nu);
        L.S32.alloc(m->N * L.nu);
      } else {
        L.T64.alloc(m->N * L.nu);
        L.S64.alloc(m->N * L.nu);
      }
      launch_fmm_leaf_T(m->N, m->d_geom.p, m->d_qidx.p, m->d_hq.p, 2 * m->g.nq, L.ec.p, L.z.p, L.s.p, L.nu, nullptr, k, FS->ra.p, FS->rb.p, FS->rw.p,
                        FS->nq, single ? nullptr : L.T64.p, single ? L.T32.p : nullptr, s);
      launch_fmm_leaf_S(m->N, m->d_geom.p, L.ec.p, L.z.p, L.s.p, L.w.p, L.nu, k, m->gre, m->gim,
                        single ? nullptr : L.S64.p, single ? L.S32.p : nullptr, s);
    }
    BEM_HIP(hipGetLastError());
    return;
  }
  FmmLevel& leaf = F->lv[nl - 1];
  if (single) {
    F->T32.alloc(m->N * leaf.nu);
    F->S32.alloc(m->N * leaf.nu);
  } else {
    F->T64.alloc(m->N * leaf.nu);
    F->S64.alloc(m->N * leaf.nu);
  }
  launch_fmm_leaf_T(m->N, m->d_geom.p, m->d_qidx.p, m->d_hq.p, 2 * m->g.nq, FS->elem_cluster.p, leaf.z.p, leaf.s.p, leaf.nu, nullptr, k, FS->ra.p, FS->rb.p,
                    FS->rw.p, FS->nq, single ? nullptr : F->T64.p, single ? F->T32.p : nullptr, s);
  launch_fmm_leaf_S(m->N, m->d_geom.p, FS->elem_cluster.p, leaf.z.p, leaf.s.p, leaf.w.p, leaf.nu, k, m->gre,
                    m->gim, single ? nullptr : F->S64.p, single ? F->S32.p : nullptr, s);
  BEM_HIP(hipGetLastError());
}

}  // namespace

void fmm_setup_problem(bem_mesh* m, hipStream_t s) {
  if (!m->fmm_state) {
    m->fmm_state = new FmmState();
    upload_tree(m, m->fmm_state, s);
  }
  FmmState* F = m->fmm_state;
  // nothing below depends on the admittance: a new beta at the same k reuses it
  if (F->k_setup == m->k && F->t_order == m->opt.t_order && F->gre_setup == m->gre && F->gim_setup == m->gim)
    return;
  F->k_setup = m->k;
  F->gre_setup = m->gre;
  F->gim_setup = m->gim;
  upload_rule(F, m->opt.t_order, s);
  if (!m->far_direct64) setup_set(m, F, 0, s);  // the FP64 far field is direct otherwise
  setup_set(m, F, 1, s);
}

void fmm_apply(bem_mesh* m, bem_op op, bem_precision prec, const double2* x, double2* y, hipStream_t s,
               bool vmode) {
  if (!m->fmm_state) throw Error(BEM_E_STATE, "FMM not set up");
  if (op == BEM_OP_A) {
    if (prec == BEM_PREC_FP64) fmm_apply_t<double, double2>(m, m->fmm_state, x, y, vmode, s);
    else fmm_apply_t<float, float2>(m, m->fmm_state, x, y, vmode, s);
  } else {
    if (prec == BEM_PREC_FP64) fmm_apply_adj_t<double, double2>(m, m->fmm_state, x, y, vmode, s);
    else fmm_apply_adj_t<float, float2>(m, m->fmm_state, x, y, vmode, s);
  }
}

size_t fmm_bytes(const bem_mesh* m) {
  const FmmState* FS = m->fmm_state;
  if (!FS) return 0;
  size_t b = 0;
  for (const FmmSet& F : FS->set) {
  b += F.T64.bytes() + F.S64.bytes() + F.T32.bytes() + F.S32.bytes();
  for (const auto& L : F.lv)
    b += L.D64.bytes() + L.D32.bytes() + L.sig64.bytes() + L.loc64.bytes() + L.sig32.bytes() + L.loc32.bytes() +
         L.shift64.bytes() + L.shift32.bytes() + L.Mi64.bytes() + L.Ma64.bytes() + L.Mi32.bytes() +
         L.Ma32.bytes() + L.MiT64.bytes() + L.MaT64.bytes() + L.MiT32.bytes() + L.MaT32.bytes() +
         L.tA64.bytes() + L.tB64.bytes() + L.tA32.bytes() + L.tB32.bytes() + L.T64.bytes() + L.S64.bytes() +
         L.T32.bytes() + L.S32.bytes() + L.ec.bytes();
  }
  return b;
}

FmmPlanInfo fmm_plan_info(const Tree& T, int64_t N, double k, const bem_options& o) {
  FmmPlanInfo I;
  const int nl = (int)T.lv.size();
  I.levels = nl;
  int top = nl - 1;
  for (int l = 0; l < nl; ++l)
    if (!T.lv[l].il.empty()) {
      top = l;
      break;
    }
  for (int l = top; l < nl && l < 16; ++l) {
    const Level& L = T.lv[l];
    double rmax = 0.0;
    for (double r : L.r) rmax = std::max(rmax, r);
    double xmin = -1.0;
    for (int64_t c = 0; c < L.nc; ++c)
      for (int64_t q = L.il_off[c]; q < L.il_off[c + 1]; ++q) {
        const int64_t n = L.il[q];
        const double d0 = L.z[3 * c] - L.z[3 * n], d1 = L.z[3 * c + 1] - L.z[3 * n + 1],
                     d2 = L.z[3 * c + 2] - L.z[3 * n + 2];
        const double v = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        if (xmin < 0.0 || v < xmin) xmin = v;
      }
    for (int single = 0; single < 2; ++single) {
      const int la = truncation_length(k, rmax, o, -1.0, single != 0);
      const int lc = truncation_length(k, rmax, o, xmin, single != 0);
      (single ? I.L32 : I.L)[l] = lc;
      if (xmin >= 0.0 && lc < la) {
        I.capped = true;
        (single ? I.capped32 : I.capped64) = true;
      }
      const double nu = 2.0 * lc * lc;
      const double b = single ? 8.0 : 16.0;
      I.bytes += b * nu * (0.5 * (double)L.il.size() + 2.0 * (double)L.nc);
      if (l == nl - 1 || (o.level_rows && !L.il.empty())) I.bytes += 2.0 * b * nu * (double)N;
    }
  }
  return I;
}


FmmLeafView fmm_leaf_view(bem_mesh* m) {
  if (!m->fmm || m->far_direct || m->far_direct64 || !m->fmm_state)
    throw Error(BEM_E_STATE, "the mesh has no FP64 FMM far field");
  FmmSet* F = &m->fmm_state->set[0];
  FmmLevel& leaf = F->lv.back();
  FmmLeafView v;
  v.L = leaf.L;
  v.nu = leaf.nu;
  v.s = leaf.s.p;
  v.w = leaf.w.p;
  v.T = F->T64.p;
  v.ebeg = m->fmm_state->leaf_ebeg.p;
  v.eend = m->fmm_state->leaf_eend.p;
  v.nc = leaf.nc;
  if (v.L <= 0) throw Error(BEM_E_STATE, "the FMM has no expansion on the leaf level");
  return v;
}

void fmm_leaf_aggregate(bem_mesh* m, const double2* x, bool factor, double2* sig, hipStream_t s) {
  const FmmLeafView v = fmm_leaf_view(m);
  FmmLevel& leaf = m->fmm_state->set[0].lv.back();
  FactorArgs fa = factor_args(m, leaf);
  fa.cfac = nullptr;
  launch_fmm_aggregate<double, double2>(v.nc, v.ebeg, v.eend, v.nu, v.T, factor ? &fa : nullptr, x, sig, false, s);
}

bool fmm_leaf_pair_stable(const bem_mesh* m, int L, double X) {
  if (m->opt.l_mode != 1) return true;  // the paper's lengths carry no stability cap
  return 2.220446049250313e-16 * (2 * L + 1) * hankel_abs(L, m->k * X) <= 0.1 * m->opt.l_eps;
}
}  // namespace bem
