// Near-field part of the Burton-Miller operator, evaluated on the fly.
//
// For every target (collocation node x_i, normal n_i) and every quadrature
// item of its near-field plan -- a (sub-)triangle of source element j with an
// order-m conical rule -- the kernel forms, at each quadrature point y,
//
//   K(x_i, y) = -(H - gamma E) + (G - gamma H') c_j          (Eq. (SystemI))
//
// with G = exp(ikr)/(4 pi r), H = dG/dn_y, H' = dG/dn_x, E = d2G/dn_x dn_y
// (Sec. 2.1, 2.5).  All four share r, 1/r and exp(ikr); with R = y - x_i,
// a = ik - 1/r and B = 3/r^2 - 3ik/r - k^2 the combination is
//
//   K = G [ -a (Rh.n_j) - gamma (B (Rh.n_i)(Rh.n_j) + a (n_i.n_j)/r) ]
//     + c_j G [ 1 + gamma a (Rh.n_i) ].
//
// Work layout: one 64-lane wavefront per target element; the target's items
// are processed one rule order at a time (uniform point loop, rule tables in
// scalar registers), lanes stride over the items of that order, each lane
// integrates its whole item and multiplies by x_j, and
// a shuffle reduction adds the lanes in a fixed order -- no atomics, so every
// run is bit-identical.  The singular self term is not an item: it is folded
// into the per-frequency diagonal A_ii (self-term kernel below).
#include "common.h"
#include "device.h"

#include <cmath>
#include <type_traits>

namespace bem {

__constant__ double c_rule_a[kRulePoints];
__constant__ double c_rule_b[kRulePoints];
__constant__ double c_rule_w[kRulePoints];
__constant__ int c_rule_off[kMaxRuleOrder + 1];
// (a, b, w / 4 pi) of every rule point in one record, for one scalar load
// per point
struct alignas(16) RulePt32 { float a, b, w, pad; };
struct alignas(32) RulePt64 { double a, b, w, pad; };
__constant__ RulePt32 c_rule_pt32[kRulePoints];
__constant__ RulePt64 c_rule_pt64[kRulePoints];
// exp(2 pi i j / kExpTab), j = 0 .. kExpTab - 1: the table of the
// table-driven exp(i theta) of the FP64 quadrature kernels (staged in LDS)
constexpr int kExpTab = 512;
__constant__ double2 c_exp_tab[kExpTab];

void upload_rule_tables(const double* a, const double* b, const double* w, const int* off) {
  // the point loops read (a, b, w / 4 pi) per point; the field kernels a, b, w
  RulePt32 pt32[kRulePoints];
  RulePt64 pt64[kRulePoints];
  for (int i = 0; i < kRulePoints; ++i) {
    const double ws = w[i] * 0.079577471545947667884441881686257181;
    pt32[i] = RulePt32{(float)a[i], (float)b[i], (float)ws, 0.0f};
    pt64[i] = RulePt64{a[i], b[i], ws, 0.0};
  }
  BEM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_rule_pt32), pt32, sizeof(pt32)));
  BEM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_rule_pt64), pt64, sizeof(pt64)));
  {
    // exp(i j 2 pi / kExpTab) from angles of at most pi/4 (within an
    // octant the argument r pi / (kExpTab / 4) carries only the rounding of
    // pi), then the exact octant and quadrant symmetries
    std::vector<double2> tab(kExpTab);
    const int quarter = kExpTab / 4;
    for (int j = 0; j < kExpTab; ++j) {
      const int q = j / quarter, r = j % quarter;
      double c, sn;
      if (2 * r <= quarter) {
        const double a = M_PI * (double)r / (double)(2 * quarter);
        c = std::cos(a);
        sn = std::sin(a);
      } else {
        const double a = M_PI * (double)(quarter - r) / (double)(2 * quarter);
        c = std::sin(a);
        sn = std::cos(a);
      }
      // rotate by q quarter turns
      for (int t = 0; t < q; ++t) {
        const double c2 = -sn;
        sn = c;
        c = c2;
      }
      tab[j] = make_double2(c, sn);
    }
    BEM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_exp_tab), tab.data(), sizeof(double2) * kExpTab));
  }
  BEM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_rule_a), a, sizeof(double) * kRulePoints));
  BEM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_rule_b), b, sizeof(double) * kRulePoints));
  BEM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_rule_w), w, sizeof(double) * kRulePoints));
  BEM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_rule_off), off, sizeof(int) * (kMaxRuleOrder + 1)));
}

namespace {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;

// field offsets (match GeomField on the host)
enum { P0X = 0, P1X = 3, P2X = 6, NX = 9, AREA = 12, CX = 13 };

template <typename T> struct RuleTab;
template <> struct RuleTab<double> {
  __device__ static RulePt64 pt(int i) { return c_rule_pt64[i]; }
};
template <> struct RuleTab<float> {
  __device__ static RulePt32 pt(int i) { return c_rule_pt32[i]; }
};

// exp(i x) for |x| < 2^20 by the table-driven method of Tang: x = j h + d
// with h = 2 pi / kExpTab and j = rint(x / h) (Cody & Waite reduction, h in
// two parts), |d| <= h / 2 = pi / 512; then exp(i x) = T[j mod kExpTab]
// exp(i d) with the Taylor series of cos d to d^4 / 4! and of sin d to
// d^5 / 5! (truncation below 7.5e-17 and 1e-20).  The table T (exp(i j h),
// computed on the host) sits in LDS.  The phases here are k r >= 0 over
// distances within a mesh, far below 2^20.
__device__ inline void cis_table(double x, const double2* __restrict__ tab, double* s, double* c) {
  constexpr double kInvH = 81.487330863050417;    // kExpTab / (2 pi)
  constexpr double kC1 = 0x1.921fb58p-7;           // 2 pi / kExpTab in two parts: kC1 has 26 significant
  constexpr double kC2 = -0x1.dde973dcb3b3ap-34;   // bits, so j kC1 is exact for |j| < 2^27; kC1 + kC2
                                                   // is within 5e-27 of 2 pi / kExpTab
  // j = nearest integer to x kInvH, read off the low word of x kInvH + 1.5 2^52
  constexpr double kRound = 0x1.8p52;
  const double jr = fma(x, kInvH, kRound);
  const double j = jr - kRound;
  const int ji = (int)(uint32_t)__builtin_bit_cast(uint64_t, jr);
  double d = fma(-j, kC1, x);
  d = fma(-j, kC2, d);
  const double2 t = tab[ji & (kExpTab - 1)];
  const double z = d * d;
  // |d| <= pi / kExpTab: cos d = 1 - z/2 + z^2/24 (the z^3 / 720 term is below
  // 7.5e-17), sin d = d (1 - z/6 + z^2/120)
  const double cd = fma(z, fma(z, 1.0 / 24.0, -0.5), 1.0);
  const double sd = fma(d * z, fma(z, 1.0 / 120.0, -1.0 / 6.0), d);
  *c = fma(t.x, cd, -t.y * sd);
  *s = fma(t.y, cd, t.x * sd);
}

// Per-block copy of the exp table into LDS (every thread of the block takes
// part; the barrier makes it visible to all of them).
__device__ inline void stage_exp_table(double2* __restrict__ lds) {
  for (int i = threadIdx.x; i < kExpTab; i += blockDim.x) lds[i] = c_exp_tab[i];
  __syncthreads();
}

// 1/sqrt(x) for positive normal x: the hardware estimate and one correction
// y (1 + e/2 + 3 e^2/8), e = 1 - x y^2 (cubic convergence; the estimate's
// relative error of order 2^-23 becomes rounding)
__device__ inline double rsqrt_t(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}
__device__ inline float rsqrt_t(float x) { return rsqrtf(x); }

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Load the (sub-)triangle of an item: element vertices, then the recorded
// sequence of child choices (children of (P0, P1, P2) with edge midpoints
// M01, M12, M20 are (P0,M01,M20), (P1,M12,M01), (P2,M20,M12), (M01,M12,M20)).
template <typename T>
__device__ inline void item_triangle(const T* __restrict__ g, int64_t N, int64_t j, int depth,
                                     uint64_t path, T v0[3], T v1[3], T v2[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    v0[c] = g[(P0X + c) * N + j];
    v1[c] = g[(P1X + c) * N + j];
    v2[c] = g[(P2X + c) * N + j];
  }
  for (int d = 0; d < depth; ++d) {
    int ch = (int)((path >> (2 * d)) & 3u);
    T m01[3], m12[3], m20[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      m01[c] = T(0.5) * (v0[c] + v1[c]);
      m12[c] = T(0.5) * (v1[c] + v2[c]);
      m20[c] = T(0.5) * (v2[c] + v0[c]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T a0, a1, a2;
      if (ch == 0) { a0 = v0[c]; a1 = m01[c]; a2 = m20[c]; }
      else if (ch == 1) { a0 = v1[c]; a1 = m12[c]; a2 = m01[c]; }
      else if (ch == 2) { a0 = v2[c]; a1 = m20[c]; a2 = m12[c]; }
      else { a0 = m01[c]; a1 = m12[c]; a2 = m20[c]; }
      v0[c] = a0; v1[c] = a1; v2[c] = a2;
    }
  }
}

// The same for integration record j: the elements' own triangles (j < N) or
// the halves of the quadrilaterals (geometry hq, stride nh).
template <typename T>
__device__ inline void rec_triangle(const T* __restrict__ g, int64_t N, const T* __restrict__ hq, int64_t nh,
                                    int64_t j, int depth, uint64_t path, T v0[3], T v1[3], T v2[3]) {
  if (j < N) item_triangle<T>(g, N, j, depth, path, v0, v1, v2);
  else item_triangle<T>(hq, nh, j - N, depth, path, v0, v1, v2);
}
// field f of integration record j
template <typename T>
__device__ inline T rec_field(const T* __restrict__ g, int64_t N, const T* __restrict__ hq, int64_t nh, int f,
                              int64_t j) {
  return j < N ? g[f * N + j] : hq[f * nh + (j - N)];
}
// element of integration record j
__device__ inline int64_t rec_owner(const QuadRecs& Q, int64_t N, int64_t j) { return j < N ? j : Q.hown[j - N]; }

// Source-element records (built per wavenumber by k_records): 16 values per
// element, all lengths multiplied by kap, the phase unit per length (k for
// radians in FP64, k/(2 pi) for revolutions in FP32):
//   v0 (3), e1 = v1 - v0 (3), e2 = v2 - v0 (3), n (3),
//   |e1|^2, |e2|^2, 2 e1.e2, 2 area.
// One element is 64 (FP32) or 128 (FP64) contiguous bytes, read with 16-byte
// loads: one gather per cache line instead of one per field.
constexpr int kRec = 16;
template <typename T> struct Rec;
template <> struct Rec<float> {
  __device__ static void load(const float* __restrict__ rec, int64_t j, float r[kRec]) {
    const float4* p = reinterpret_cast<const float4*>(rec) + 4 * j;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 v = p[q];
      r[4 * q] = v.x;
      r[4 * q + 1] = v.y;
      r[4 * q + 2] = v.z;
      r[4 * q + 3] = v.w;
    }
  }
};
template <> struct Rec<double> {
  __device__ static void load(const double* __restrict__ rec, int64_t j, double r[kRec]) {
    const double2* p = reinterpret_cast<const double2*>(rec) + 8 * j;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double2 v = p[q];
      r[2 * q] = v.x;
      r[2 * q + 1] = v.y;
    }
  }
};

// Per-launch constants of the point loop (see integrate_item), from the
// wavenumber k, the scale kap and the coupling gamma = gre + i gim.
template <typename T> struct PointConsts {
  T kr;                      // k / kap
  T kgr, kgi;                // kap gamma
  T Q0r, Q0i, Q1r, Q1i, Q2r, Q2i;
  T ikap;                    // 1 / kap
  const double2* ex;         // FP64: the exp table in LDS (see cis_table)
};
// exp of the phase in the unit the kernels use: radians in FP64 (table
// driven), revolutions in FP32 (the hardware sine and cosine take
// revolutions, so k/(2 pi) is folded into the per-item constants)
__device__ inline void phase_cis(const PointConsts<double>& P, double x, double* s, double* c) {
  cis_table(x, P.ex, s, c);
}
__device__ inline void phase_cis(const PointConsts<float>& P, float x, float* s, float* c) {
  *s = __builtin_amdgcn_sinf(x);
  *c = __builtin_amdgcn_cosf(x);
}
template <typename T>
__device__ inline PointConsts<T> point_consts(double k, double kap, double gre, double gim) {
  PointConsts<T> P;
  const double k2 = k * k / (3.0 * kap);
  P.kr = (T)(k / kap);
  P.kgr = (T)(kap * gre);
  P.kgi = (T)(kap * gim);
  P.Q0r = (T)(gre * k2);  // gamma k^2 / (3 kap)
  P.Q0i = (T)(gim * k2);
  P.Q1r = (T)(-gim * k);  // i gamma k
  P.Q1i = (T)(gre * k);
  P.Q2r = (T)(-gre * kap);  // -gamma kap
  P.Q2i = (T)(-gim * kap);
  P.ikap = (T)(1.0 / kap);
  P.ex = nullptr;
  return P;
}

// The constants and, for FP64, the exp table staged in the block's LDS
// (lds: a __shared__ array of kExpTab entries, used only when T is double;
// every thread of the block must call this)
template <typename T>
__device__ inline PointConsts<T> point_consts_staged(double k, double kap, double gre, double gim, double2* lds) {
  PointConsts<T> P = point_consts<T>(k, kap, gre, gim);
  if constexpr (sizeof(T) == sizeof(double)) {
    stage_exp_table(lds);
    P.ex = lds;
  }
  return P;
}

// Integrate one item: returns S1 (c-independent part) and S2 (c_j part),
// both already multiplied by 2 * area of the (sub-)triangle.
// m is the item's rule order; the caller passes it wavefront-uniform so the
// rule tables are read with scalar loads.  S1: the c-independent part
// -(H - gamma E); S2: the part multiplied by c_j, (G - gamma H').
// xs: the collocation point times kap; ni its normal.
// With d0 = v0 - x_i and the point y = v0 + a e1 + b e2 in the (flat) source
// triangle, everything the kernels need is a low-order polynomial in (a, b)
// with per-item coefficients: |y - x|^2 is a quadratic form, (y - x).n_j = d0.n_j
// (e1, e2 lie in the source plane) and (y - x).n_i = cx is affine.
// Written in u = 1/r, with H = hn + gamma nn (hn = (y - x).n_j, nn = n_i.n_j)
// and sigma = 3 hn cx, the two integrands (weight w, kernel e^{ikr}/(4 pi r))
// collapse to
//   S1:  w e^{ikr} u^2 [-ik H + u (H + sigma gamma (k^2/3 + iku - u^2))],
//   S2:  w e^{ikr} u   [1 + cx u gamma (ik - u)].
// The loop runs on the kap-scaled geometry of the records, in U = 1/(kap r):
// the phase is kap r = r2 U with r2 the scaled quadratic form, and with
// primes for scaled lengths (hn' = kap hn, cx' = kap cx, H' = kap H,
// sigma' = 3 hn' cx', area' = kap^2 area)
//   S1 = w e^{i theta} U^2 [Hk + U (H' + sigma' (Q0 + U (Q1 + U Q2)))] 2 area',
//   S2 = w e^{i theta} U   [1 + cx' U (Q1 + U Q2)] 2 area' / kap,
// Hk = -i (k/kap) H', Q0 = gamma k^2/(3 kap), Q1 = i gamma k, Q2 = -gamma kap.
// Sub-triangles are formed in edge form: the children (P0, M01, M20),
// (P1, M12, M01), (P2, M20, M12), (M01, M12, M20) of (P0, P1, P2), with
// midpoints M, have v0 = P0, P1, P2, M01 and edges that are halves of
// +-e1, +-e2, e2 - e1.
// integrate_loaded: the same with the source's record r already in registers.
// ONEPT: evaluate one-point items at the point itself (the direct far field,
// where they are common; elsewhere the general loop handles them and the
// kernel keeps fewer registers)
template <typename T, bool WANT_S1, bool WANT_S2, bool ONEPT = false>
__device__ inline void integrate_loaded(const T r[kRec], uint64_t item, int m, const T xs[3], const T ni[3],
                                        const PointConsts<T>& P, T& s1r, T& s1i, T& s2r, T& s2i) {
  const int depth = (int)((item >> 29) & 15u);
  const uint64_t path = item >> 33;
  T v0[3] = {r[0], r[1], r[2]}, e1[3] = {r[3], r[4], r[5]}, e2[3] = {r[6], r[7], r[8]};
  const T nj[3] = {r[9], r[10], r[11]};
  T q11 = r[12], q22 = r[13], q12 = r[14], area2 = r[15];
  if (depth > 0) {
    for (int d = 0; d < depth; ++d) {
      const int ch = (int)((path >> (2 * d)) & 3u);
      // v0 += al e1 + be e2; (e1, e2) <- (a11 e1 + a12 e2, a21 e1 + a22 e2)
      const T al = ch == 1 ? T(1) : (ch == 3 ? T(0.5) : T(0));
      const T be = ch == 2 ? T(1) : T(0);
      const T a11 = ch == 0 ? T(0.5) : (ch == 1 ? T(-0.5) : T(0));
      const T a12 = ch == 0 ? T(0) : (ch == 2 ? T(-0.5) : T(0.5));
      const T a21 = ch == 0 ? T(0) : (ch == 2 ? T(0.5) : T(-0.5));
      const T a22 = ch == 1 ? T(0) : (ch == 2 ? T(-0.5) : T(0.5));
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T f1 = e1[c], f2 = e2[c];
        v0[c] = fma(al, f1, fma(be, f2, v0[c]));
        e1[c] = fma(a11, f1, a12 * f2);
        e2[c] = fma(a21, f1, a22 * f2);
      }
    }
    q11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    q22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    q12 = T(2) * (e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]);
    area2 = ldexp(area2, -2 * depth);
  }
  const T nn = ni[0] * nj[0] + ni[1] * nj[1] + ni[2] * nj[2];
  T d0[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) d0[c] = v0[c] - xs[c];
  if (ONEPT && m == 1) {
    // one rule point: the integrand at y itself, without the quadratic-form
    // coefficients
    const auto rp = RuleTab<T>::pt(c_rule_off[0]);
    T d[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c] = fma(rp.a, e1[c], fma(rp.b, e2[c], d0[c]));
    const T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const T U = rsqrt_t(r2);
    T sn, cs;
    phase_cis(P, r2 * U, &sn, &cs);
    const T hn = d[0] * nj[0] + d[1] * nj[1] + d[2] * nj[2];
    const T cx = d[0] * ni[0] + d[1] * ni[1] + d[2] * ni[2];
    const T Rr = fma(U, P.Q2r, P.Q1r), Ri = fma(U, P.Q2i, P.Q1i);
    const T qwU = rp.w * U;
    T a1r = 0, a1i = 0, a2r = 0, a2i = 0;
    if (WANT_S1) {
      const T sg = T(3) * hn * cx;
      const T Hr = fma(P.kgr, nn, hn), Hi = P.kgi * nn;
      const T Wr = fma(sg, fma(U, Rr, P.Q0r), Hr);
      const T Wi = fma(sg, fma(U, Ri, P.Q0i), Hi);
      const T Vr = fma(U, Wr, P.kr * Hi), Vi = fma(U, Wi, -P.kr * Hr);
      const T g2 = qwU * U;
      const T Gr = g2 * cs, Gi = g2 * sn;
      a1r = fma(Gr, Vr, -Gi * Vi);
      a1i = fma(Gr, Vi, Gi * Vr);
    }
    if (WANT_S2) {
      const T cU = cx * U;
      const T Zr = fma(cU, Rr, T(1)), Zi = cU * Ri;
      const T Gr = qwU * cs, Gi = qwU * sn;
      a2r = fma(Gr, Zr, -Gi * Zi);
      a2i = fma(Gr, Zi, Gi * Zr);
    }
    const T f2 = area2 * P.ikap;
    s1r = a1r * area2;
    s1i = a1i * area2;
    s2r = a2r * f2;
    s2i = a2i * f2;
    return;
  }
  // |d0 + a e1 + b e2|^2 = q00 + a (qa1 + a q11) + b (qb1 + b q22 + a q12)
  const T q00 = d0[0] * d0[0] + d0[1] * d0[1] + d0[2] * d0[2];
  const T qa1 = T(2) * (d0[0] * e1[0] + d0[1] * e1[1] + d0[2] * e1[2]);
  const T qb1 = T(2) * (d0[0] * e2[0] + d0[1] * e2[1] + d0[2] * e2[2]);
  // hn = (y - x).n_j; cx = (y - x).n_i = c0 + a c1 + b c2
  const T hn = d0[0] * nj[0] + d0[1] * nj[1] + d0[2] * nj[2];
  T c0 = d0[0] * ni[0] + d0[1] * ni[1] + d0[2] * ni[2];
  T c1 = e1[0] * ni[0] + e1[1] * ni[1] + e1[2] * ni[2];
  T c2 = e2[0] * ni[0] + e2[1] * ni[1] + e2[2] * ni[2];
  const T h3 = T(3) * hn;
  if (!WANT_S2) {
    // only sigma is needed: fold 3 hn into the affine coefficients
    c0 *= h3;
    c1 *= h3;
    c2 *= h3;
  }
  const T Hr = fma(P.kgr, nn, hn), Hi = P.kgi * nn;
  const T Hkr = P.kr * Hi, Hki = -P.kr * Hr;
  const int base = c_rule_off[m - 1];
  const int np = m * m;
  T a1r = 0, a1i = 0, a2r = 0, a2i = 0;
#pragma unroll 2
  for (int q = 0; q < np; ++q) {
    // (a, b, w) of the point in one scalar load
    const auto rp = RuleTab<T>::pt(base + q);
    const T qa = rp.a, qb = rp.b, qw = rp.w;
    const T ta = fma(qa, q11, qa1);
    T tb = fma(qb, q22, qb1);
    tb = fma(qa, q12, tb);
    T r2 = fma(qa, ta, q00);
    r2 = fma(qb, tb, r2);
    const T U = rsqrt_t(r2);
    T sn, cs;
    phase_cis(P, r2 * U, &sn, &cs);
    // cx, or sigma when S2 is not wanted
    const T cx = fma(qb, c2, fma(qa, c1, c0));
    const T Rr = fma(U, P.Q2r, P.Q1r), Ri = fma(U, P.Q2i, P.Q1i);
    const T qwU = qw * U;
    if (WANT_S1) {
      const T sg = WANT_S2 ? h3 * cx : cx;
      const T Wr = fma(sg, fma(U, Rr, P.Q0r), Hr);
      const T Wi = fma(sg, fma(U, Ri, P.Q0i), Hi);
      const T Vr = fma(U, Wr, Hkr), Vi = fma(U, Wi, Hki);
      const T g2 = qwU * U;
      const T Gr = g2 * cs, Gi = g2 * sn;
      a1r = fma(Gr, Vr, fma(-Gi, Vi, a1r));
      a1i = fma(Gr, Vi, fma(Gi, Vr, a1i));
    }
    if (WANT_S2) {
      const T cU = cx * U;
      const T Zr = fma(cU, Rr, T(1)), Zi = cU * Ri;
      const T Gr = qwU * cs, Gi = qwU * sn;
      a2r = fma(Gr, Zr, fma(-Gi, Zi, a2r));
      a2i = fma(Gr, Zi, fma(Gi, Zr, a2i));
    }
  }
  const T f2 = area2 * P.ikap;
  s1r = a1r * area2;
  s1i = a1i * area2;
  s2r = a2r * f2;
  s2i = a2i * f2;
}

template <typename T, bool WANT_S1, bool WANT_S2, bool ONEPT = false>
__device__ inline void integrate_item(const T* __restrict__ rec, uint64_t item, int m, const T xs[3],
                                      const T ni[3], const PointConsts<T>& P, T& s1r, T& s1i, T& s2r,
                                      T& s2i, int64_t& jout) {
  const int64_t j = (int64_t)(item & ((uint64_t(1) << 26) - 1));
  jout = j;
  T r[kRec];
  Rec<T>::load(rec, j, r);
  integrate_loaded<T, WANT_S1, WANT_S2, ONEPT>(r, item, m, xs, ni, P, s1r, s1i, s2r, s2i);
}

template <typename T> __device__ inline const T* near_rec(const NearLaunch& L);
template <> __device__ inline const double* near_rec<double>(const NearLaunch& L) { return L.rec; }
template <> __device__ inline const float* near_rec<float>(const NearLaunch& L) { return L.rec32; }
template <typename T> __device__ inline double near_kap(const NearLaunch& L);
template <> __device__ inline double near_kap<double>(const NearLaunch& L) { return L.kap; }
template <> __device__ inline double near_kap<float>(const NearLaunch& L) { return L.kap32; }

// One pipeline slot of the forward kernel: an item and what its source
// contributes besides the rule (record, x_j, c_j).
template <typename T> struct Slot {
  uint64_t item;
  T r[kRec];
  double2 x, c;
};
template <typename T, bool NEED_C>
__device__ inline void load_slot(const NearLaunch& L, const T* __restrict__ rec, const double2* __restrict__ x,
                                 uint64_t item, Slot<T>& S) {
  const int64_t j = (int64_t)(item & ((uint64_t(1) << 26) - 1));
  S.item = item;
  Rec<T>::load(rec, j, S.r);
  const int64_t o = rec_owner(L.Q, L.N, j);  // the element whose unknown the record carries
  S.x = x[o];
  if (NEED_C) S.c = L.cfac[o];
}
// acc += K_ij x_j (VMODE: the dA/dc entry) for the slot's item
template <typename T, bool HAS_C, bool VMODE>
__device__ inline void accumulate_slot(const Slot<T>& S, int m, const T xs[3], const T ni[3],
                                       const PointConsts<T>& P, T& accr, T& acci) {
  T s1r, s1i, s2r, s2i;
  integrate_loaded<T, !VMODE, HAS_C || VMODE>(S.r, S.item, m, xs, ni, P, s1r, s1i, s2r, s2i);
  T vr = s1r, vi = s1i;
  if (VMODE) {
    vr = s2r;
    vi = s2i;
  } else if (HAS_C) {
    const T cr = (T)S.c.x, ci = (T)S.c.y;
    vr += cr * s2r - ci * s2i;
    vi += cr * s2i + ci * s2r;
  }
  const T xr = (T)S.x.x, xim = (T)S.x.y;
  accr += vr * xr - vi * xim;
  acci += vr * xim + vi * xr;
}

// VMODE: apply dA/dc -- the (G - gamma H') part without c_j, diagonal
// G_ii - gamma/2 -- instead of A.
// WPB wavefronts per workgroup; the launch shape is a tuning choice.  With
// one wavefront per target the grid covers all targets; a smaller grid
// (L.nwaves) keeps its wavefronts resident and each loops over the targets
// w, w + stride, ..., leaving wavefront slots to kernels that run beside it.
template <typename T, bool HAS_C, bool VMODE, int WPB = 4>
__global__ __launch_bounds__(64 * WPB) void k_near(NearLaunch L, const T* __restrict__ g,
                                                   const double2* __restrict__ x, double2* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t N = L.N;
  const double kap = near_kap<T>(L);
  const T* __restrict__ rec = near_rec<T>(L);
  __shared__ double2 s_ex[sizeof(T) == sizeof(double) ? kExpTab : 1];
  const PointConsts<T> P = point_consts_staged<T>(L.k, kap, L.gre, L.gim, s_ex);
  constexpr bool NEED_C = HAS_C && !VMODE;
  const int64_t stride = (int64_t)gridDim.x * WPB;
  // the target is uniform across the wavefront: say so, so that its data go
  // through scalar loads and registers.  Targets are visited in L.order
  // (groups of decreasing work), so the last wavefronts to start are short ones.
  // this launch's share of the targets: positions first .. first + count of
  // the visiting order (count 0: all)
  const int64_t cnt = L.count > 0 ? L.count : N;
  for (int64_t w = (int64_t)blockIdx.x * WPB + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); w < cnt;
       w += stride) {
    const int64_t t = L.order ? (int64_t)L.order[L.first + w] : L.first + w;
    T xs[3], ni[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xs[c] = (T)(kap * L.geom[(CX + c) * N + t]);
      ni[c] = g[(NX + c) * N + t];
    }
    T accr = 0, acci = 0;
    // the target's items are sorted by rule order; seg[t][m-1] .. seg[t][m]
    // holds the order-m items, so every pass below runs one uniform rule
    const int64_t* sg = L.seg + t * (kMaxRuleOrder + 1);
    for (int mc = 0; mc < kMaxRuleOrder; ++mc) {
      const int64_t b = sg[mc], e = sg[mc + 1];
      if (b == e) continue;
      // passes of 64 items; each pass loads the next pass's item (index
      // clamped into the segment) before integrating its own
      const int64_t npass = (e - b + 63) >> 6;
      const int64_t last = e - 1;
      int64_t it = b + lane;
      uint64_t item = L.items[it < last ? it : last];
      for (int64_t p = 0; p < npass; ++p, it += 64) {
        const uint64_t next = L.items[it + 64 < last ? it + 64 : last];
        if (it < e) {
          Slot<T> S;
          load_slot<T, NEED_C>(L, rec, x, item, S);
          accumulate_slot<T, HAS_C, VMODE>(S, mc + 1, xs, ni, P, accr, acci);
        }
        item = next;
      }
    }
    double sr = wave_sum((double)accr);
    double si = wave_sum((double)acci);
    if (lane == 0) {
      const double2 d = VMODE ? L.vdiag[t] : L.diag[t];
      const double2 xt = x[t];
      y[t] = make_double2(d.x * xt.x - d.y * xt.y + sr, d.x * xt.y + d.y * xt.x + si);
    }
  }
}

// Conjugate transpose: items are indexed by source j ("targets" of this
// launch are sources); the item's element field holds the collocation index i.
// y_j = conj(A_jj) x_j + sum_i conj(K_ij) x_i.
template <typename T, bool HAS_C, bool VMODE>
__global__ __launch_bounds__(256) void k_near_adj(NearLaunch L, const T* __restrict__ g,
                                                  const double2* __restrict__ x, double2* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t jsrc = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const double kap = near_kap<T>(L);
  __shared__ double2 s_ex[sizeof(T) == sizeof(double) ? kExpTab : 1];
  const PointConsts<T> P = point_consts_staged<T>(L.k, kap, L.gre, L.gim, s_ex);  // whole block, before any exit
  if (jsrc >= L.N) return;
  const int64_t N = L.N;
  const T* __restrict__ rec = near_rec<T>(L);
  T cr = 0, ci = 0;
  if (HAS_C) {
    const double2 c = L.cfac[jsrc];
    cr = (T)c.x;
    ci = (T)c.y;
  }
  T accr = 0, acci = 0;
  // a quadrilateral's items name their half in bit 63
  const int64_t qj = L.Q.nh ? L.Q.qidx[jsrc] : -1;
  const int64_t* sg = L.seg + jsrc * (kMaxRuleOrder + 1);
  for (int mc = 0; mc < kMaxRuleOrder; ++mc) {
    const int64_t b = sg[mc], e = sg[mc + 1];
    if (b == e) continue;
    for (int64_t it = b + lane; it < e; it += 64) {
      const uint64_t raw = L.items[it];
      const int64_t i = (int64_t)(raw & ((uint64_t(1) << 26) - 1));
      // rebuild the forward item (source record of jsrc) and integrate from target i
      const int64_t recj = qj >= 0 ? N + 2 * qj + (int64_t)(raw >> 63) : jsrc;
      const uint64_t item = (raw & ~((uint64_t(1) << 26) - 1) & ~(uint64_t(1) << 63)) | (uint64_t)recj;
      T xs[3], ni[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        xs[c] = (T)(kap * L.geom[(CX + c) * N + i]);
        ni[c] = g[(NX + c) * N + i];
      }
      T s1r, s1i, s2r, s2i;
      int64_t jj;
      integrate_item<T, !VMODE, HAS_C || VMODE>(rec, item, mc + 1, xs, ni, P, s1r, s1i, s2r, s2i, jj);
      T vr = s1r, vi = s1i;
      if (VMODE) {
        vr = s2r;
        vi = s2i;
      } else if (HAS_C) {
        vr += cr * s2r - ci * s2i;
        vi += cr * s2i + ci * s2r;
      }
      const double2 xv = x[i];
      const T xr = (T)xv.x, xim = (T)xv.y;
      // conj(v) * x
      accr += vr * xr + vi * xim;
      acci += vr * xim - vi * xr;
    }
  }
  double sr = wave_sum((double)accr);
  double si = wave_sum((double)acci);
  if (lane == 0) {
    const double2 d = VMODE ? L.vdiag[jsrc] : L.diag[jsrc];
    const double2 xt = x[jsrc];
    y[jsrc] = make_double2(d.x * xt.x + d.y * xt.y + sr, d.x * xt.y - d.y * xt.x + si);
  }
}

template <typename T, int WPB>
void near_forward(const NearLaunch& L, const T* g, const double2* x, double2* y, hipStream_t s) {
  const int64_t cnt = L.count > 0 ? L.count : L.N;
  const int64_t waves = L.nwaves > 0 && L.nwaves < cnt ? L.nwaves : cnt;
  dim3 grid((unsigned)((waves + WPB - 1) / WPB)), block(64 * WPB);
  if (L.cfac) hipLaunchKernelGGL((k_near<T, true, false, WPB>), grid, block, 0, s, L, g, x, y);
  else hipLaunchKernelGGL((k_near<T, false, false, WPB>), grid, block, 0, s, L, g, x, y);
}

template <typename T>
void near_dispatch(const NearLaunch& L, const T* g, const double2* x, double2* y, hipStream_t s, bool adj,
                   bool vmode) {
  if (L.N <= 0) return;
  dim3 grid((unsigned)((L.N + 3) / 4)), block(256);
  if (vmode) {
    if (!adj) hipLaunchKernelGGL((k_near<T, false, true>), grid, block, 0, s, L, g, x, y);
    else hipLaunchKernelGGL((k_near_adj<T, false, true>), grid, block, 0, s, L, g, x, y);
  } else if (!adj) {
    switch (L.wpb) {
      case 1: near_forward<T, 1>(L, g, x, y, s); break;
      case 2: near_forward<T, 2>(L, g, x, y, s); break;
      case 8: near_forward<T, 8>(L, g, x, y, s); break;
      default: near_forward<T, 4>(L, g, x, y, s); break;
    }
  } else {
    if (L.cfac) hipLaunchKernelGGL((k_near_adj<T, true, false>), grid, block, 0, s, L, g, x, y);
    else hipLaunchKernelGGL((k_near_adj<T, false, false>), grid, block, 0, s, L, g, x, y);
  }
}

// ------------------------------------------------------ element records ---
// Records of the integration kernels (layout at Rec above), FP64 with scale
// kap and FP32 with scale kap32; the scaled quantities are formed in FP64.
__global__ __launch_bounds__(256) void k_records(int64_t N, const double* __restrict__ g, int64_t first,
                                                 double kap, double kap32, double* __restrict__ rec,
                                                 float* __restrict__ rec32) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  double v0[3], e1[3], e2[3], n[3];
  for (int c = 0; c < 3; ++c) {
    v0[c] = g[(P0X + c) * N + t];
    e1[c] = g[(P1X + c) * N + t] - v0[c];
    e2[c] = g[(P2X + c) * N + t] - v0[c];
    n[c] = g[(NX + c) * N + t];
  }
  const double area = g[AREA * N + t];
  for (int p = 0; p < 2; ++p) {
    const double s = p == 0 ? kap : kap32;
    double r[kRec], f1[3], f2[3];
    for (int c = 0; c < 3; ++c) {
      r[c] = s * v0[c];
      f1[c] = s * e1[c];
      f2[c] = s * e2[c];
      r[3 + c] = f1[c];
      r[6 + c] = f2[c];
      r[9 + c] = n[c];
    }
    r[12] = f1[0] * f1[0] + f1[1] * f1[1] + f1[2] * f1[2];
    r[13] = f2[0] * f2[0] + f2[1] * f2[1] + f2[2] * f2[2];
    r[14] = 2.0 * (f1[0] * f2[0] + f1[1] * f2[1] + f1[2] * f2[2]);
    r[15] = 2.0 * area * s * s;
    for (int q = 0; q < kRec; ++q) {
      if (p == 0) rec[kRec * (first + t) + q] = r[q];
      else rec32[kRec * (first + t) + q] = (float)r[q];
    }
  }
}

// ------------------------------------------------------------ self terms ---
// G_ii by the Duffy rule on the sub-triangles that join the collocation node
// to the vertices and edge midpoints (Sec. 3.1.1: six on a triangle, eight on
// a quadrilateral); E_ii = sum over the counter-clockwise edges of
// int (n x grad_y G) . dy plus k^2 G_ii (Sec. 3.1.2); H_ii = H'_ii = 0.  Then
// A_ii = (1 - gamma c_i)/2 + gamma E_ii + G_ii c_i.
// Duffy and edge sums of one element with NV vertices P (lanes share the points)
template <int NV>
__device__ inline void self_sums(const SelfLaunch& L, const double (&P)[4][3], const double x[3], const double n[3],
                                 int lane, double& Gr, double& Gi, double& Er, double& Ei) {
  const double k = L.k;
  double M[NV][3];
#pragma unroll
  for (int e = 0; e < NV; ++e)
    for (int c = 0; c < 3; ++c) M[e][c] = 0.5 * (P[e][c] + P[(e + 1) % NV][c]);
  // Duffy triangles (V[h], V[h + 1]) with V = P0, M01, P1, M12, P2, ...
  const double* V[2 * NV];
#pragma unroll
  for (int e = 0; e < NV; ++e) {
    V[2 * e] = P[e];
    V[2 * e + 1] = M[e];
  }
  const int nn2 = L.self_n * L.self_n;
#pragma unroll
  for (int h = 0; h < 2 * NV; ++h) {
    const double* Q1 = V[h];
    const double* Q2 = V[(h + 1) % (2 * NV)];
    double a[3], b[3], d[3];
    for (int c = 0; c < 3; ++c) {
      a[c] = Q1[c] - x[c];
      b[c] = Q2[c] - x[c];
      d[c] = Q2[c] - Q1[c];
    }
    const double cr[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    const double As2 = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    for (int pnt = lane; pnt < nn2; pnt += 64) {
      const int ia = pnt / L.self_n, ib = pnt - ia * L.self_n;
      const double u = L.duffy_u[ia], wu = L.duffy_w[ia];
      const double v = L.duffy_u[ib], wv = L.duffy_w[ib];
      double R[3];
      for (int c = 0; c < 3; ++c) R[c] = u * (a[c] + v * d[c]);
      const double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
      double sn, cs;
      sincos(k * r, &sn, &cs);
      const double wgt = As2 * u * wu * wv * kInv4Pi / r;
      Gr += wgt * cs;
      Gi += wgt * sn;
    }
  }
  // edges P_e -> P_(e+1): (n x R) . d with grad_y G = G (ik - 1/r) R / r
#pragma unroll
  for (int e = 0; e < NV; ++e) {
    const double* Pa = P[e];
    const double* Pb = P[(e + 1) % NV];
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = Pb[c] - Pa[c];
    for (int q = lane; q < L.edge_pts; q += 64) {
      double R[3];
      for (int c = 0; c < 3; ++c) R[c] = Pa[c] + L.edge_t[q] * d[c] - x[c];
      const double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
      const double rinv = 1.0 / r;
      double sn, cs;
      sincos(k * r, &sn, &cs);
      const double nxR[3] = {n[1] * R[2] - n[2] * R[1], n[2] * R[0] - n[0] * R[2], n[0] * R[1] - n[1] * R[0]};
      const double proj = nxR[0] * d[0] + nxR[1] * d[1] + nxR[2] * d[2];
      const double s = L.edge_w[q] * proj * kInv4Pi * rinv * rinv;
      // exp(ikr) (ik - 1/r) = (cs + i sn)(-1/r + i k)
      Er += s * (-cs * rinv - sn * k);
      Ei += s * (cs * k - sn * rinv);
    }
  }
}

__global__ __launch_bounds__(256) void k_self(SelfLaunch L, double2* __restrict__ diag) {
  // one wavefront per element; lanes share the element's quadrature points
  // (the Duffy triangles' self_n^2 points each, then the edge points)
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (t >= L.N) return;
  const int64_t N = L.N;
  const double* g = L.geom;
  const int64_t q = L.Q.nh ? L.Q.qidx[t] : -1;
  double P[4][3], x[3], n[3];
  for (int v = 0; v < 3; ++v)
    for (int c = 0; c < 3; ++c) P[v][c] = g[(P0X + 3 * v + c) * N + t];
  // a quadrilateral's P3 is the last vertex of its second half
  for (int c = 0; c < 3; ++c) P[3][c] = q >= 0 ? L.Q.hq[(P2X + c) * L.Q.nh + 2 * q + 1] : P[2][c];
  for (int c = 0; c < 3; ++c) {
    x[c] = g[(CX + c) * N + t];
    n[c] = g[(NX + c) * N + t];
  }
  const double k = L.k;
  double Gr = 0, Gi = 0, Er = 0, Ei = 0;
  if (q >= 0)  // wavefront-uniform
    self_sums<4>(L, P, x, n, lane, Gr, Gi, Er, Ei);
  else
    self_sums<3>(L, P, x, n, lane, Gr, Gi, Er, Ei);
  Gr = wave_sum(Gr);
  Gi = wave_sum(Gi);
  Er = wave_sum(Er);
  Ei = wave_sum(Ei);
  if (lane != 0) return;
  Er += k * k * Gr;
  Ei += k * k * Gi;
  double cr = 0, ci = 0;
  if (L.cfac) {
    cr = L.cfac[t].x;
    ci = L.cfac[t].y;
  }
  // (1 - gamma c)/2 + gamma E + G c
  const double gcr = L.gre * cr - L.gim * ci, gci = L.gre * ci + L.gim * cr;
  double dr = 0.5 * (1.0 - gcr) + (L.gre * Er - L.gim * Ei) + (Gr * cr - Gi * ci);
  double di = -0.5 * gci + (L.gre * Ei + L.gim * Er) + (Gr * ci + Gi * cr);
  diag[t] = make_double2(dr, di);
  // dA/dc on the diagonal: G_ii - gamma/2
  if (L.vdiag) L.vdiag[t] = make_double2(Gr - 0.5 * L.gre, Gi - 0.5 * L.gim);
}




// ----------------------------------------------- direct far field (no FMM) ---
template <typename T>
__device__ inline const T* far_geom(const FarLaunch& F);
template <>
__device__ inline const double* far_geom<double>(const FarLaunch& F) { return F.geom; }
template <>
__device__ inline const float* far_geom<float>(const FarLaunch& F) { return F.geom32; }
template <typename T> __device__ inline const T* far_rec(const FarLaunch& F);
template <> __device__ inline const double* far_rec<double>(const FarLaunch& F) { return F.rec; }
template <> __device__ inline const float* far_rec<float>(const FarLaunch& F) { return F.rec32; }
template <typename T> __device__ inline const T* far_hq(const FarLaunch& F);
template <> __device__ inline const double* far_hq<double>(const FarLaunch& F) { return F.Q.hq; }
template <> __device__ inline const float* far_hq<float>(const FarLaunch& F) { return F.Q.hq32; }
template <typename T> __device__ inline double far_kap(const FarLaunch& F);
template <> __device__ inline double far_kap<double>(const FarLaunch& F) { return F.kap; }
template <> __device__ inline double far_kap<float>(const FarLaunch& F) { return F.kap32; }

// order for r~^2 (0: split)
// r~^2 = d2 / area, compared as d2 against threshold * area (no division);
// the complex-FP32 kernels take their own thresholds
template <typename T>
__device__ inline int far_order(const FarLaunch& F, double d2, double area) {
  const double* th = sizeof(T) == 4 ? F.rt2_min32 : F.rt2_min;
  if (d2 < F.ratio2 * area) return 0;
  for (int m = 1; m <= F.m_max; ++m)
    if (d2 > th[m - 1] * area) return m;
  return F.split_on_cap ? 0 : F.m_max;
}

// One (collocation i, integration record j) pair that needs subdivision:
// depth-first walk over (depth, path) without a stack, per-sub-triangle rule
// as in the plan.  The rule choice uses the unscaled geometry (g, or the
// quadrilaterals' halves), the integration the records.
template <typename T, bool WANT_S1, bool WANT_S2, bool QUADS>
__device__ void far_pair_split(const FarLaunch& F, const T* g, const T* rec, int64_t j, const T xi[3],
                               const T xs[3], const T ni[3], const PointConsts<T>& P, T& s1r, T& s1i, T& s2r,
                               T& s2i) {
  const int64_t N = F.N;
  const T* hq = far_hq<T>(F);
  const double area0 = QUADS ? (double)rec_field<T>(g, N, hq, F.Q.nh, AREA, j) : (double)g[AREA * N + j];
  int depth = 0;
  uint64_t path = 0;
  s1r = s1i = s2r = s2i = T(0);
  for (;;) {
    T v0[3], v1[3], v2[3];
    if (QUADS)
      rec_triangle<T>(g, N, hq, F.Q.nh, j, depth, path, v0, v1, v2);
    else
      item_triangle<T>(g, N, j, depth, path, v0, v1, v2);
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double dc = (double)xi[c] - ((double)v0[c] + (double)v1[c] + (double)v2[c]) / 3.0;
      d2 += dc * dc;
    }
    const double area = area0 * ldexp(1.0, -2 * depth);
    int m = far_order<T>(F, d2, area);
    if (m == 0 && depth < F.max_subdiv && depth < 15) {
      ++depth;
      continue;
    }
    if (m == 0) m = F.m_max;  // depth limit: the plan refuses such meshes, never reached
    const uint64_t item = (uint64_t)j | ((uint64_t)depth << 29) | (path << 33);
    T a1r, a1i, a2r, a2i;
    int64_t jj;
    integrate_item<T, WANT_S1, WANT_S2, true>(rec, item, m, xs, ni, P, a1r, a1i, a2r, a2i, jj);
    s1r += a1r;
    s1i += a1i;
    s2r += a2r;
    s2i += a2i;
    while (depth > 0) {
      const int sh = 2 * (depth - 1);
      if (((path >> sh) & 3u) < 3u) {
        path += (uint64_t)1 << sh;
        break;
      }
      path &= ~((uint64_t)3 << sh);
      --depth;
    }
    if (depth == 0) break;
  }
}

// One wavefront per row r: forward r = collocation point i, lanes over far
// source elements j; adjoint r = source element j, lanes over far collocation
// points i (the far relation of leaf clusters is symmetric).  QUADS: the mesh
// has quadrilaterals, whose two integration records are taken in turn (a
// separate instantiation, so that triangle meshes keep the smaller register
// footprint of one record per pair).
template <typename T, bool HAS_C, bool VMODE, bool ADJ, bool QUADS>
__global__ __launch_bounds__(256) void k_far_direct(FarLaunch F, const double2* __restrict__ x,
                                                    double2* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const double kap = far_kap<T>(F);
  __shared__ double2 s_ex[sizeof(T) == sizeof(double) ? kExpTab : 1];
  const PointConsts<T> P = point_consts_staged<T>(F.k, kap, F.gre, F.gim, s_ex);  // whole block, before any exit
  if (r >= F.N) return;
  const int64_t N = F.N;
  const T* g = far_geom<T>(F);
  const T* __restrict__ rec = far_rec<T>(F);
  T xr[3], nr[3], xsr[3];
  for (int c = 0; c < 3; ++c) {
    xr[c] = g[(CX + c) * N + r];
    nr[c] = g[(NX + c) * N + r];
    xsr[c] = (T)(kap * F.geom[(CX + c) * N + r]);
  }
  T cr = 0, ci = 0;
  if (ADJ && HAS_C) {
    const double2 c = F.cfac[r];
    cr = (T)c.x;
    ci = (T)c.y;
  }
  const int leaf = F.elem_leaf[r];
  T accr = 0, acci = 0;
  for (int64_t q = F.far_off[leaf]; q < F.far_off[leaf + 1]; ++q) {
    const int64_t e = F.far_end[q];
    for (int64_t base = F.far_beg[q]; base < e; base += 64) {
      const int64_t o = base + lane;  // the other element of the pair
      const bool valid = o < e;
      const int64_t oi = valid ? o : r;
      // collocation point and element of this lane's pair
      const int64_t i = ADJ ? oi : r;
      const int64_t j = ADJ ? r : oi;
      T xi[3], ni[3], xs[3];
      for (int c = 0; c < 3; ++c) {
        xi[c] = ADJ ? g[(CX + c) * N + i] : xr[c];
        ni[c] = ADJ ? g[(NX + c) * N + i] : nr[c];
        xs[c] = ADJ ? (T)(kap * F.geom[(CX + c) * N + i]) : xsr[c];
      }
      T s1r = 0, s1i = 0, s2r = 0, s2i = 0;
      if constexpr (QUADS) {
        // the element's integration records: itself, or a quadrilateral's halves
        const int64_t qj = valid ? F.Q.qidx[j] : -1;
        for (int h = 0; h < 2; ++h) {
          if (h == 1 && __ballot(qj >= 0) == 0) break;
          const int64_t rj = qj >= 0 ? F.N + 2 * qj + h : j;
          const bool act = valid && (h == 0 || qj >= 0);
          int m = -1;
          if (act) {
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
              const double dc = (double)xi[c] - (double)rec_field<T>(g, N, far_hq<T>(F), F.Q.nh, CX + c, rj);
              d2 += dc * dc;
            }
            m = far_order<T>(F, d2, (double)rec_field<T>(g, N, far_hq<T>(F), F.Q.nh, AREA, rj));
          }
          T a1r = 0, a1i = 0, a2r = 0, a2i = 0;
          // one uniform rule per pass
          for (int mc = 1; mc <= kMaxRuleOrder; ++mc) {
            if (__ballot(m == mc) == 0) continue;
            if (m == mc) {
              int64_t jj;
              integrate_item<T, !VMODE, HAS_C || VMODE, true>(rec, (uint64_t)rj, mc, xs, ni, P, a1r, a1i, a2r, a2i,
                                                             jj);
            }
          }
          if (__ballot(m == 0) != 0 && m == 0)
            far_pair_split<T, !VMODE, HAS_C || VMODE, true>(F, g, rec, rj, xi, xs, ni, P, a1r, a1i, a2r, a2i);
          s1r += a1r;
          s1i += a1i;
          s2r += a2r;
          s2i += a2i;
        }
      } else {
        int m = -1;
        if (valid) {
          double d2 = 0.0;
          for (int c = 0; c < 3; ++c) {
            const double dc = (double)xi[c] - (double)g[(CX + c) * N + j];
            d2 += dc * dc;
          }
          m = far_order<T>(F, d2, (double)g[AREA * N + j]);
        }
        // one uniform rule per pass
        for (int mc = 1; mc <= kMaxRuleOrder; ++mc) {
          if (__ballot(m == mc) == 0) continue;
          if (m == mc) {
            int64_t jj;
            integrate_item<T, !VMODE, HAS_C || VMODE, true>(rec, (uint64_t)j, mc, xs, ni, P, s1r, s1i, s2r, s2i,
                                                           jj);
          }
        }
        if (__ballot(m == 0) != 0 && m == 0)
          far_pair_split<T, !VMODE, HAS_C || VMODE, false>(F, g, rec, j, xi, xs, ni, P, s1r, s1i, s2r, s2i);
      }
      if (!valid) continue;
      T vr = s1r, vi = s1i;
      if (VMODE) {
        vr = s2r;
        vi = s2i;
      } else if (HAS_C) {
        T ccr = cr, cci = ci;
        if (!ADJ) {
          const double2 c = F.cfac[j];
          ccr = (T)c.x;
          cci = (T)c.y;
        }
        vr += ccr * s2r - cci * s2i;
        vi += ccr * s2i + cci * s2r;
      }
      const double2 xv = x[oi];
      const T xa = (T)xv.x, xb = (T)xv.y;
      if (ADJ) {
        accr += vr * xa + vi * xb;
        acci += vr * xb - vi * xa;
      } else {
        accr += vr * xa - vi * xb;
        acci += vr * xb + vi * xa;
      }
    }
  }
  const double sr = wave_sum((double)accr);
  const double si = wave_sum((double)acci);
  if (lane == 0) {
    const double2 yo = y[r];
    y[r] = make_double2(yo.x + sr, yo.y + si);
  }
}

// The forward direct far field on triangle meshes with several collocation
// points per wavefront: the points of one group (up to G consecutive points
// of one leaf cluster, F.grp) share the far list of their leaf, so each
// source element's record, centre, area and x_j are loaded once per pass and
// integrated against every point of the group.  Each point's contributions
// arrive in the same order as in k_far_direct (the results agree to
// rounding: the compiler may contract the two kernels differently); the
// loads per pair drop G-fold (the one-point-per-wavefront kernel is bound by
// the L2 traffic of these loads in FP64).
template <typename T, bool HAS_C, bool VMODE, int G>
__global__ __launch_bounds__(256) void k_far_rows(FarLaunch F, const double2* __restrict__ x,
                                                  double2* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const double kap = far_kap<T>(F);
  __shared__ double2 s_ex[sizeof(T) == sizeof(double) ? kExpTab : 1];
  const PointConsts<T> P = point_consts_staged<T>(F.k, kap, F.gre, F.gim, s_ex);  // whole block, before any exit
  if (w >= F.ngrp) return;
  const int64_t N = F.N;
  const T* g = far_geom<T>(F);
  const T* __restrict__ rec = far_rec<T>(F);
  const int64_t code = F.grp[w];
  const int64_t r0 = code >> 3;
  const int nr = (int)(code & 7) + 1;  // points in the group, 1..G
  const int leaf = F.elem_leaf[r0];
  // per-lane partial sums of the group's points, lane-private in LDS (the
  // point loop then needs no unrolling and the kernel no register array)
  using V2 = typename std::conditional<sizeof(T) == sizeof(double), double2, float2>::type;
  __shared__ V2 s_acc[4][G][64];
  V2* acc = &s_acc[threadIdx.x >> 6][0][lane];
  for (int u = 0; u < G; ++u) {
    acc[64 * u].x = T(0);
    acc[64 * u].y = T(0);
  }
  for (int64_t q = F.far_off[leaf]; q < F.far_off[leaf + 1]; ++q) {
    const int64_t e = F.far_end[q];
    for (int64_t base = F.far_beg[q]; base < e; base += 64) {
      const int64_t o = base + lane;
      const bool valid = o < e;
      const int64_t j = valid ? o : r0;
      T rj[kRec];
      Rec<T>::load(rec, j, rj);
      const double cj0 = (double)g[CX * N + j], cj1 = (double)g[(CX + 1) * N + j], cj2 = (double)g[(CX + 2) * N + j];
      const double aj = (double)g[AREA * N + j];
      const double2 xv = x[j];
      T ccr = 0, cci = 0;
      if (HAS_C && !VMODE) {
        const double2 c = F.cfac[j];
        ccr = (T)c.x;
        cci = (T)c.y;
      }
#pragma unroll 1
      for (int u = 0; u < nr; ++u) {
        const int64_t r = r0 + u;
        T xi[3], ni[3], xs[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          xi[c] = g[(CX + c) * N + r];
          ni[c] = g[(NX + c) * N + r];
          xs[c] = (T)(kap * F.geom[(CX + c) * N + r]);
        }
        int m = -1;
        if (valid) {
          const double d0 = (double)xi[0] - cj0, d1 = (double)xi[1] - cj1, d2c = (double)xi[2] - cj2;
          double d2 = 0.0;
          d2 += d0 * d0;
          d2 += d1 * d1;
          d2 += d2c * d2c;
          m = far_order<T>(F, d2, aj);
        }
        T s1r = 0, s1i = 0, s2r = 0, s2i = 0;
        for (int mc = 1; mc <= kMaxRuleOrder; ++mc) {
          if (__ballot(m == mc) == 0) continue;
          if (m == mc)
            integrate_loaded<T, !VMODE, HAS_C || VMODE, true>(rj, (uint64_t)j, mc, xs, ni, P, s1r, s1i, s2r, s2i);
        }
        if (__ballot(m == 0) != 0 && m == 0)
          far_pair_split<T, !VMODE, HAS_C || VMODE, false>(F, g, rec, j, xi, xs, ni, P, s1r, s1i, s2r, s2i);
        if (valid) {
          T vr = s1r, vi = s1i;
          if (VMODE) {
            vr = s2r;
            vi = s2i;
          } else if (HAS_C) {
            vr += ccr * s2r - cci * s2i;
            vi += ccr * s2i + cci * s2r;
          }
          const T xa = (T)xv.x, xb = (T)xv.y;
          T ar = acc[64 * u].x, ai = acc[64 * u].y;
          ar += vr * xa - vi * xb;
          ai += vr * xb + vi * xa;
          acc[64 * u].x = ar;
          acc[64 * u].y = ai;
        }
      }
    }
  }
  for (int u = 0; u < nr; ++u) {
    const double sr = wave_sum((double)acc[64 * u].x);
    const double si = wave_sum((double)acc[64 * u].y);
    if (lane == 0) {
      const double2 yo = y[r0 + u];
      y[r0 + u] = make_double2(yo.x + sr, yo.y + si);
    }
  }
}

// ------------------------------------------------ preconditioner blocks ---
// One wavefront per row t: the row's near items whose source lies in t's block
// (B.items: a compact per-row list built with the blocks) are integrated (FP64)
// and summed per column in a fixed order (lane order of the item chunks), so
// the assembly is deterministic; lane jl owns column jl.
template <bool HAS_C>
__global__ __launch_bounds__(256) void k_block_assemble(NearLaunch L, BlockArgs B, double2* __restrict__ a) {
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __shared__ double2 s_ex[kExpTab];
  const PointConsts<double> P = point_consts_staged<double>(L.k, L.kap, L.gre, L.gim, s_ex);  // before any exit
  if (t >= L.N) return;
  const int64_t N = L.N;
  const double* g = L.geom;
  const int blk = B.elem_blk[t];
  const int64_t b0 = B.beg[blk];
  const int n = B.n[blk];
  const int64_t off = B.off[blk];
  const int il = (int)(t - b0);
  double xs[3], ni[3];
  for (int c = 0; c < 3; ++c) {
    xs[c] = L.kap * g[(CX + c) * N + t];
    ni[c] = g[(NX + c) * N + t];
  }
  double accr = 0.0, acci = 0.0;
  const int64_t* sg = B.seg + t * (kMaxRuleOrder + 1);
  for (int mc = 0; mc < kMaxRuleOrder; ++mc) {
    const int64_t e = sg[mc + 1];
    for (int64_t base = sg[mc]; base < e; base += 64) {
      const int64_t it = base + lane;
      int64_t j = -1;
      bool in = false;
      if (it < e) {
        j = rec_owner(L.Q, N, (int64_t)(B.items[it] & ((uint64_t(1) << 26) - 1)));
        in = j >= b0 && j < b0 + n;
      }
      double vr = 0.0, vi = 0.0;
      if (in) {
        double s1r, s1i, s2r, s2i;
        int64_t jj;
        integrate_item<double, true, HAS_C>(L.rec, B.items[it], mc + 1, xs, ni, P, s1r, s1i, s2r,
                                            s2i, jj);
        vr = s1r;
        vi = s1i;
        if (HAS_C) {
          const double2 c = L.cfac[j];
          vr += c.x * s2r - c.y * s2i;
          vi += c.x * s2i + c.y * s2r;
        }
      }
      uint64_t mask = __ballot(in);
      const int jl = in ? (int)(j - b0) : -1;
      while (mask) {
        const int src = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        const int cj = __shfl(jl, src);
        const double wr = __shfl(vr, src), wi = __shfl(vi, src);
        if (lane == cj) {
          accr += wr;
          acci += wi;
        }
      }
    }
  }
  if (lane == il) {
    accr += L.diag[t].x;
    acci += L.diag[t].y;
  }
  if (lane < n) a[off + (int64_t)lane * n + il] = make_double2(accr, acci);
}

// ------------------------------------------------------------ field points ---
// Exterior field (Eq. (BIE_I) with lambda = 1): K_fj = I^H(x_f, G_j) - c_j I^G(x_f, G_j)
// with the quasi-singular / regular rules of Sec. 3.1.3-3.1.4 chosen on the fly
// from r~ = |x_f - mid| / sqrt(A): split while r~ < ratio, else the estimator
// order, capped or split as for the collocation plan.  The subdivision tree is
// walked depth first without a stack: (depth, path) names the current
// sub-triangle with the same child numbering as the near-field items.
__device__ inline int field_order(double rt, double eps) {
  const double q = 1.0 / (2.0 * rt);
  for (int m = 1; m <= 64; ++m) {
    const double eg = 32.0 * pow(q, (double)(2 * m + 1));
    const double eh = 64.0 * (double)(2 * m + 1) * pow(q, (double)(2 * m + 2));
    const double ee = 128.0 * (double)(m + 1) * (double)(2 * m + 1) * pow(q, (double)(2 * m + 3));
    if (eg < eps && eh < eps && ee < eps) return m;
  }
  return 64;
}

// integrals (I^G, I^H) of integration record j (normal nj) seen from x,
// added to gr, gi, hr, hi; false on a subdivision overflow
__device__ bool field_record(const FieldArgs& A, int64_t j, const double nj[3], const double x[3], double& gr,
                             double& gi, double& hr, double& hi) {
  const int64_t N = A.N;
  const double* g = A.geom;
  const double area0 = rec_field<double>(g, N, A.Q.hq, A.Q.nh, AREA, j);
  const int max_depth = A.max_subdiv < 15 ? A.max_subdiv : 15;
  int depth = 0;
  uint64_t path = 0;
  for (;;) {
    double v0[3], v1[3], v2[3];
    rec_triangle<double>(g, N, A.Q.hq, A.Q.nh, j, depth, path, v0, v1, v2);
    const double area = area0 * ldexp(1.0, -2 * depth);
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double dc = x[c] - (v0[c] + v1[c] + v2[c]) / 3.0;
      d2 += dc * dc;
    }
    const double rt = sqrt(d2) / sqrt(area);
    bool split = rt < A.ratio;
    int m = 1;
    if (!split) {
      m = field_order(rt, A.eps);
      if (m > A.m_max) {
        if (A.split_on_cap) split = true;
        else m = A.m_max;
      }
    }
    if (split) {
      if (depth >= max_depth) return false;
      ++depth;  // first child: digit 0
      continue;
    }
    const int base = c_rule_off[m - 1];
    double e1[3], e2[3];
    for (int c = 0; c < 3; ++c) {
      e1[c] = v1[c] - v0[c];
      e2[c] = v2[c] - v0[c];
    }
    double sgr = 0, sgi = 0, shr = 0, shi = 0;
    for (int q = 0; q < m * m; ++q) {
      const double qa = c_rule_a[base + q], qb = c_rule_b[base + q], qw = c_rule_w[base + q];
      double R[3];
      for (int c = 0; c < 3; ++c) R[c] = (v0[c] + qa * e1[c] + qb * e2[c]) - x[c];
      const double r2 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2];
      const double rinv = rsqrt(r2);
      double sn, cs;
      sincos(A.k * (r2 * rinv), &sn, &cs);
      const double gs = qw * rinv * kInv4Pi;
      const double Gr = gs * cs, Gi = gs * sn;
      const double rny = (R[0] * nj[0] + R[1] * nj[1] + R[2] * nj[2]) * rinv;
      // H = G (ik - 1/r) rny
      sgr += Gr;
      sgi += Gi;
      shr += (-Gr * rinv - Gi * A.k) * rny;
      shi += (Gr * A.k - Gi * rinv) * rny;
    }
    const double a2 = 2.0 * area;
    gr += a2 * sgr;
    gi += a2 * sgi;
    hr += a2 * shr;
    hi += a2 * shi;
    // next sub-triangle in depth-first order
    while (depth > 0) {
      const int sh = 2 * (depth - 1);
      if (((path >> sh) & 3u) < 3u) {
        path += (uint64_t)1 << sh;
        break;
      }
      path &= ~((uint64_t)3 << sh);
      --depth;
    }
    if (depth == 0) break;
  }
  return true;
}

// integrals (I^G, I^H) of element j seen from x (both halves of a
// quadrilateral); false on a subdivision overflow
__device__ bool field_integrals(const FieldArgs& A, int64_t j, const double x[3], double2& IG, double2& IH) {
  const int64_t N = A.N;
  const double* g = A.geom;
  const double nj[3] = {g[(NX + 0) * N + j], g[(NX + 1) * N + j], g[(NX + 2) * N + j]};
  double gr = 0, gi = 0, hr = 0, hi = 0;
  const int64_t q = A.Q.nh ? A.Q.qidx[j] : -1;
  if (q < 0) {
    if (!field_record(A, j, nj, x, gr, gi, hr, hi)) return false;
  } else {
    for (int h = 0; h < 2; ++h)
      if (!field_record(A, N + 2 * q + h, nj, x, gr, gi, hr, hi)) return false;
  }
  IG = make_double2(gr, gi);
  IH = make_double2(hr, hi);
  return true;
}

// p_out[f] = p_inc[f] + sum_j K_fj p[j]  (one wavefront per field point)
__global__ __launch_bounds__(256) void k_field(FieldArgs A, const double* __restrict__ pts,
                                               const double2* __restrict__ p, const double2* __restrict__ pinc,
                                               double2* __restrict__ out, int64_t* __restrict__ err) {
  const int lane = threadIdx.x & 63;
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (f >= A.npts) return;
  const double x[3] = {pts[3 * f], pts[3 * f + 1], pts[3 * f + 2]};
  double ar = 0, ai = 0;
  for (int64_t j = lane; j < A.N; j += 64) {
    double2 IG, IH;
    if (!field_integrals(A, j, x, IG, IH)) {
      err[0] = j;
      continue;
    }
    const double2 pj = p[j];
    if (A.dpdn) {
      // tau (I^H p_j - I^G (dp/dn)_j) with the normal derivative given
      const double2 vj = A.dpdn[j];
      ar += A.tau * ((IH.x * pj.x - IH.y * pj.y) - (IG.x * vj.x - IG.y * vj.y));
      ai += A.tau * ((IH.x * pj.y + IH.y * pj.x) - (IG.x * vj.y + IG.y * vj.x));
      continue;
    }
    double kr = IH.x, ki = IH.y;
    if (A.cfac && A.part == 0) {
      const double2 c = A.cfac[j];
      kr -= c.x * IG.x - c.y * IG.y;
      ki -= c.x * IG.y + c.y * IG.x;
    }
    if (A.part == 1) {
      kr = IG.x;
      ki = IG.y;
    }
    ar += kr * pj.x - ki * pj.y;
    ai += kr * pj.y + ki * pj.x;
  }
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  if (lane == 0) {
    const double2 b = pinc ? pinc[f] : make_double2(0.0, 0.0);
    out[f] = make_double2(b.x + ar, b.y + ai);
  }
}

// Evaluation grid, one wavefront per point f (points in cluster order, point
// cluster pc[f] with centre zp):
//   out[f] = pinc[f] + tau ( near + far ),
//   near = sum over the elements j of the cluster's near leaf clusters of
//          I^H_j(x) p_j - I^G_j(x) v_j (same rules as k_field),
//   far  = -(ik / 16 pi^2) sum_nu w_nu exp(ik (x - zp).s_nu) loc[pc][nu].
__global__ __launch_bounds__(256) void k_grid_eval(FieldArgs A, int64_t npts, const double* __restrict__ pts,
                                                   const int64_t* __restrict__ pc, const double* __restrict__ zp,
                                                   int nu, const double* __restrict__ sn, const double* __restrict__ wn,
                                                   const double2* __restrict__ loc,
                                                   const int64_t* __restrict__ near_off,
                                                   const int64_t* __restrict__ near_beg,
                                                   const int64_t* __restrict__ near_end,
                                                   const double2* __restrict__ p, const double2* __restrict__ v,
                                                   const double2* __restrict__ pinc, double2* __restrict__ out,
                                                   int64_t* __restrict__ err) {
  const int lane = threadIdx.x & 63;
  const int64_t f = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (f >= npts) return;
  const double x[3] = {pts[3 * f], pts[3 * f + 1], pts[3 * f + 2]};
  const int64_t c = pc[f];
  const double d0 = x[0] - zp[3 * c], d1 = x[1] - zp[3 * c + 1], d2 = x[2] - zp[3 * c + 2];
  double fr = 0.0, fi = 0.0;
  for (int q = lane; q < nu; q += 64) {
    double snv, csv;
    sincos(A.k * (d0 * sn[3 * q] + d1 * sn[3 * q + 1] + d2 * sn[3 * q + 2]), &snv, &csv);
    const double2 l = loc[c * nu + q];
    const double w = wn[q];
    fr += w * (csv * l.x - snv * l.y);
    fi += w * (csv * l.y + snv * l.x);
  }
  // -(ik / 16 pi^2) (fr + i fi)
  constexpr double kInv16Pi2 = 0.0063325739776461107152;
  double ar = A.k * kInv16Pi2 * fi, ai = -A.k * kInv16Pi2 * fr;
  for (int64_t r = near_off[c]; r < near_off[c + 1]; ++r)
    for (int64_t j = near_beg[r] + lane; j < near_end[r]; j += 64) {
      double2 IG, IH;
      if (!field_integrals(A, j, x, IG, IH)) {
        err[0] = j;
        continue;
      }
      const double2 pj = p[j], vj = v[j];
      ar += (IH.x * pj.x - IH.y * pj.y) - (IG.x * vj.x - IG.y * vj.y);
      ai += (IH.x * pj.y + IH.y * pj.x) - (IG.x * vj.y + IG.y * vj.x);
    }
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  if (lane == 0) {
    const double2 b = pinc ? pinc[f] : make_double2(0.0, 0.0);
    out[f] = make_double2(b.x + A.tau * ar, b.y + A.tau * ai);
  }
}

// v = c p elementwise (the normal derivative of admittance / sound-hard elements)
__global__ void k_cmul(int64_t N, const double2* __restrict__ c, const double2* __restrict__ p, double2* __restrict__ v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double2 a = c ? c[t] : make_double2(0.0, 0.0), b = p[t];
  v[t] = make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// y[j] = sum_f conj(K_fj) g[f]  (one wavefront per element); part 1: K = I^G
__global__ __launch_bounds__(256) void k_field_adj(FieldArgs A, const double* __restrict__ pts,
                                                   const double2* __restrict__ gv, double2* __restrict__ y,
                                                   int64_t* __restrict__ err) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= A.N) return;
  double ar = 0, ai = 0;
  double cr = 0, ci = 0;
  if (A.cfac && A.part == 0) {
    cr = A.cfac[j].x;
    ci = A.cfac[j].y;
  }
  for (int64_t f = lane; f < A.npts; f += 64) {
    const double x[3] = {pts[3 * f], pts[3 * f + 1], pts[3 * f + 2]};
    double2 IG, IH;
    if (!field_integrals(A, j, x, IG, IH)) {
      err[0] = j;
      continue;
    }
    double kr, ki;
    if (A.part == 1) {
      kr = IG.x;
      ki = IG.y;
    } else {
      kr = IH.x - (cr * IG.x - ci * IG.y);
      ki = IH.y - (cr * IG.y + ci * IG.x);
    }
    const double2 gf = gv[f];
    // conj(K) g
    ar += kr * gf.x + ki * gf.y;
    ai += kr * gf.y - ki * gf.x;
  }
  ar = wave_sum(ar);
  ai = wave_sum(ai);
  if (lane == 0) y[j] = make_double2(ar, ai);
}

// energy[0] = sum_f |p_f|^2 (one block)
__global__ __launch_bounds__(256) void k_energy(int64_t n, const double2* __restrict__ p, double* __restrict__ energy) {
  __shared__ double part[4];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) acc += p[i].x * p[i].x + p[i].y * p[i].y;
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) energy[0] = (part[0] + part[1]) + (part[2] + part[3]);
}

// grad[e] = 2 Re{ dc p_e (-conj(w_e) - conj(hg_e)) },  dc = -i k rho_c
// (caller order; the derivative of sum_f |p_f|^2 with respect to Y_e, with
// beta = rho_c Y; w = V^H mu from the adjoint solve, hg = (I^G)^H p_field)
__global__ void k_grad_admittance(int64_t N, double k, double rho_c, const double2* __restrict__ p,
                                  const double2* __restrict__ w, const double2* __restrict__ hg,
                                  double* __restrict__ grad) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  const double2 pe = p[e], we = w[e], he = hg[e];
  // t = -conj(w) - conj(hg)
  const double tr = -we.x - he.x, ti = we.y + he.y;
  // u = p_e t
  const double ur = pe.x * tr - pe.y * ti, ui = pe.x * ti + pe.y * tr;
  // Re{ -i k rho_c u } = k rho_c Im(u)
  grad[e] = 2.0 * k * rho_c * ui;
}

// -------------------------------------------------------- small kernels ---
__global__ void k_rhs_plane(int64_t N, const double* __restrict__ g, double k, double gre, double gim,
                            double d0, double d1, double d2, double p0r, double p0i, double2* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double ph = k * (g[CX * N + t] * d0 + g[(CX + 1) * N + t] * d1 + g[(CX + 2) * N + t] * d2);
  double sn, cs;
  sincos(ph, &sn, &cs);
  const double pr = p0r * cs - p0i * sn, pi = p0r * sn + p0i * cs;
  const double dn = k * (g[NX * N + t] * d0 + g[(NX + 1) * N + t] * d1 + g[(NX + 2) * N + t] * d2);
  // dp/dn = i dn p ; b = p - gamma dp/dn
  const double qr = -dn * pi, qi = dn * pr;
  out[t] = make_double2(pr - (gre * qr - gim * qi), pi - (gre * qi + gim * qr));
}

__global__ void k_rhs_point(int64_t N, const double* __restrict__ g, double k, double gre, double gim,
                            double s0, double s1, double s2, double p0r, double p0i, double2* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double R0 = g[CX * N + t] - s0, R1 = g[(CX + 1) * N + t] - s1, R2 = g[(CX + 2) * N + t] - s2;
  const double R = sqrt(R0 * R0 + R1 * R1 + R2 * R2);
  double sn, cs;
  sincos(k * R, &sn, &cs);
  const double sc = kInv4Pi / R;
  const double pr = sc * (p0r * cs - p0i * sn), pi = sc * (p0r * sn + p0i * cs);
  const double rn = (R0 * g[NX * N + t] + R1 * g[(NX + 1) * N + t] + R2 * g[(NX + 2) * N + t]) / R;
  // dp/dn = p (ik - 1/R) rn
  const double fr = -rn / R, fi = k * rn;
  const double qr = pr * fr - pi * fi, qi = pr * fi + pi * fr;
  out[t] = make_double2(pr - (gre * qr - gim * qi), pi - (gre * qi + gim * qr));
}

// incident pressure at arbitrary points: kind 0 plane wave along s, kind 1
// point source at s (Sec. 2.4)
__global__ void k_incident(int64_t n, const double* __restrict__ pts, int kind, double k, double s0, double s1,
                           double s2, double p0r, double p0i, double2* __restrict__ out) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n) return;
  const double x0 = pts[3 * f], x1 = pts[3 * f + 1], x2 = pts[3 * f + 2];
  double ph, sc = 1.0;
  if (kind == 0) {
    ph = k * (x0 * s0 + x1 * s1 + x2 * s2);
  } else {
    const double R0 = x0 - s0, R1 = x1 - s1, R2 = x2 - s2;
    const double R = sqrt(R0 * R0 + R1 * R1 + R2 * R2);
    ph = k * R;
    sc = kInv4Pi / R;
  }
  double sn, cs;
  sincos(ph, &sn, &cs);
  out[f] = make_double2(sc * (p0r * cs - p0i * sn), sc * (p0r * sn + p0i * cs));
}

__global__ void k_gather(int64_t N, const int64_t* __restrict__ perm, const double2* __restrict__ src,
                         double2* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) dst[t] = src[perm[t]];
}

__global__ void k_scatter(int64_t N, const int64_t* __restrict__ perm, const double2* __restrict__ src,
                          double2* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < N) dst[perm[t]] = src[t];
}

__global__ void k_cfac(int64_t N, const int64_t* __restrict__ perm, const double2* __restrict__ beta,
                       double k, double2* __restrict__ cf) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double2 b = beta[perm[t]];
  // c = -i k beta (k carries the sign -tau: +i |k| beta on interior problems)
  cf[t] = make_double2(k * b.y, -k * b.x);
}

__global__ void k_velocity(int64_t N, const double2* __restrict__ beta, double inv_rc,
                           const double2* __restrict__ p, double2* __restrict__ v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const double2 b = beta ? beta[t] : make_double2(0.0, 0.0);
  const double2 q = p[t];
  v[t] = make_double2(-inv_rc * (b.x * q.x - b.y * q.y), -inv_rc * (b.x * q.y + b.y * q.x));
}

// PRES elements (tree position t, caller index perm[t]): the solution holds
// dp/dn there, so the normal particle velocity is dp/dn / (i w rho) =
// -i (dp/dn) / (k rho_c)
__global__ void k_velocity_pres(int64_t N, const int64_t* __restrict__ perm, const double* __restrict__ pres,
                                double scale, const double2* __restrict__ p, double2* __restrict__ v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N || pres[t] == 0.0) return;
  const int64_t e = perm[t];
  const double2 q = p[e];
  v[e] = make_double2(scale * q.y, -scale * q.x);
}

inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_near(const NearLaunch& L, bool fp64, bool adjoint, bool vmode, const double2* x, double2* y,
                 hipStream_t s) {
  if (fp64) near_dispatch<double>(L, L.geom, x, y, s, adjoint, vmode);
  else near_dispatch<float>(L, L.geom32, x, y, s, adjoint, vmode);
}

void launch_records(int64_t N, const double* geom, double kap, double kap32, double* rec, float* rec32,
                    hipStream_t s) {
  launch_records_at(N, geom, 0, kap, kap32, rec, rec32, s);
}

void launch_records_at(int64_t n, const double* geom, int64_t first, double kap, double kap32, double* rec,
                       float* rec32, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_records, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, geom, first, kap, kap32, rec,
                     rec32);
}

void launch_self_terms(const SelfLaunch& L, double2* diag, hipStream_t s) {
  if (L.N <= 0) return;
  hipLaunchKernelGGL(k_self, dim3(blocks_for(L.N, 4)), dim3(256), 0, s, L, diag);
}

void launch_rhs_plane(int64_t N, const double* geom, double k, double gre, double gim, const double* d,
                      double p0re, double p0im, double2* out, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_rhs_plane, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, geom, k, gre, gim,
                     d[0], d[1], d[2], p0re, p0im, out);
}

void launch_rhs_point(int64_t N, const double* geom, double k, double gre, double gim, const double* x0,
                      double p0re, double p0im, double2* out, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_rhs_point, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, geom, k, gre, gim,
                     x0[0], x0[1], x0[2], p0re, p0im, out);
}

void launch_incident(int64_t n, const double* pts, int kind, double k, const double* src, double p0re,
                     double p0im, double2* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_incident, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, pts, kind, k, src[0], src[1],
                     src[2], p0re, p0im, out);
}

void launch_gather(int64_t N, const int64_t* perm, const double2* src, double2* dst, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, perm, src, dst);
}

void launch_scatter(int64_t N, const int64_t* perm, const double2* src, double2* dst, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, perm, src, dst);
}

void launch_cfac(int64_t N, const int64_t* perm, const double2* beta, double k, double2* cf,
                 hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_cfac, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, perm, beta, k, cf);
}

void launch_field(const FieldArgs& A, const double* pts, const double2* p, const double2* pinc, double2* out,
                  int64_t* err, hipStream_t s) {
  if (A.npts <= 0) return;
  hipLaunchKernelGGL(k_field, dim3(blocks_for(A.npts, 4)), dim3(256), 0, s, A, pts, p, pinc, out, err);
}

template <typename T, bool HAS_C, bool VMODE, bool ADJ>
void far_launch_t(const FarLaunch& F, const double2* x, double2* y, hipStream_t s) {
  if (!ADJ && !F.Q.nh && F.grp && F.ngrp > 0) {
    hipLaunchKernelGGL((k_far_rows<T, HAS_C, VMODE, kFarRows>), dim3(blocks_for(F.ngrp, 4)), dim3(256), 0, s, F, x,
                       y);
    return;
  }
  if (F.Q.nh)
    hipLaunchKernelGGL((k_far_direct<T, HAS_C, VMODE, ADJ, true>), dim3(blocks_for(F.N, 4)), dim3(256), 0, s, F, x, y);
  else
    hipLaunchKernelGGL((k_far_direct<T, HAS_C, VMODE, ADJ, false>), dim3(blocks_for(F.N, 4)), dim3(256), 0, s, F, x,
                       y);
}

template <typename T>
void far_launch_p(const FarLaunch& F, bool adjoint, bool vmode, const double2* x, double2* y, hipStream_t s) {
  const bool c = F.cfac != nullptr;
  if (vmode) {
    if (adjoint) far_launch_t<T, false, true, true>(F, x, y, s);
    else far_launch_t<T, false, true, false>(F, x, y, s);
  } else if (c) {
    if (adjoint) far_launch_t<T, true, false, true>(F, x, y, s);
    else far_launch_t<T, true, false, false>(F, x, y, s);
  } else {
    if (adjoint) far_launch_t<T, false, false, true>(F, x, y, s);
    else far_launch_t<T, false, false, false>(F, x, y, s);
  }
}

void launch_far_direct(const FarLaunch& F, bool fp64, bool adjoint, bool vmode, const double2* x, double2* y,
                       hipStream_t s) {
  if (F.N <= 0) return;
  if (fp64) far_launch_p<double>(F, adjoint, vmode, x, y, s);
  else far_launch_p<float>(F, adjoint, vmode, x, y, s);
}

void launch_block_assemble(const NearLaunch& L, const BlockArgs& B, double2* a, hipStream_t s) {
  if (L.N <= 0) return;
  if (L.cfac)
    hipLaunchKernelGGL(k_block_assemble<true>, dim3(blocks_for(L.N, 4)), dim3(256), 0, s, L, B, a);
  else
    hipLaunchKernelGGL(k_block_assemble<false>, dim3(blocks_for(L.N, 4)), dim3(256), 0, s, L, B, a);
}

void launch_grid_eval(const FieldArgs& A, const double* pts, const int64_t* pc, const double* zp, int nu,
                      const double* sn, const double* wn, const double2* loc, const int64_t* near_off,
                      const int64_t* near_beg, const int64_t* near_end, const double2* p, const double2* v,
                      const double2* pinc, double2* out, int64_t* err, hipStream_t s) {
  if (A.npts <= 0) return;
  hipLaunchKernelGGL(k_grid_eval, dim3(blocks_for(A.npts, 4)), dim3(256), 0, s, A, A.npts, pts, pc, zp, nu, sn, wn,
                     loc, near_off, near_beg, near_end, p, v, pinc, out, err);
}

void launch_cmul(int64_t N, const double2* c, const double2* p, double2* v, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_cmul, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, c, p, v);
}

void launch_energy(int64_t n, const double2* p, double* energy, hipStream_t s) {
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, s, n, p, energy);
}

void launch_field_adj(const FieldArgs& A, const double* pts, const double2* g, double2* y, int64_t* err,
                      hipStream_t s) {
  if (A.N <= 0) return;
  hipLaunchKernelGGL(k_field_adj, dim3(blocks_for(A.N, 4)), dim3(256), 0, s, A, pts, g, y, err);
}

void launch_grad_admittance(int64_t N, double k, double rho_c, const double2* p, const double2* w,
                            const double2* hg, double* grad, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_grad_admittance, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, k, rho_c, p, w, hg, grad);
}

void launch_velocity(int64_t N, const double2* beta, double rho_c, const double2* p, double2* v,
                     hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_velocity, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, beta, 1.0 / rho_c, p, v);
}

void launch_velocity_pres(int64_t N, const int64_t* perm, const double* pres, double k, double rho_c,
                          const double2* p, double2* v, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_velocity_pres, dim3(blocks_for(N, 256)), dim3(256), 0, s, N, perm, pres, 1.0 / (k * rho_c),
                     p, v);
}

}  // namespace bem
