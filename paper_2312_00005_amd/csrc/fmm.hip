// Multilevel FMM far field on the cluster tree (Sec. 3.3).
//
// Per application:
//   leaf aggregation   Sig_c(nu) = sum_{j in c} T'[j][nu] x_j
//   upward pass        Sig_p = sum_children shift_c * Interp(Sig_c)
//   translation        Loc_m(nu) = sum_{n in IL(m)} D[m,n][nu] Sig_n(nu)     (every level)
//   downward pass      Loc_c += Anterp(conj(shift_c) * Loc_p)
//   disaggregation     y_i += sum_nu S'[i][nu] Loc_c(i)(nu)
// with T' (element integral of the outgoing plane wave times the combined
// source factor c_j + ik s.n_j) and S' (quadrature weight, ik/(16 pi^2) and
// the target factor 1 - gamma ik s.n_i) precomputed per frequency.
//
// Interpolation between a child grid (L_c) and a parent grid (L_p) is the
// band-limited resampling in spherical harmonics of degree < L_c, factored
// into an azimuthal DFT, one dense (L_p x L_c) matrix per azimuthal order and
// an inverse DFT; anterpolation is its weighted transpose.  When the grids
// coincide only the shift is applied.
//
// Every output element has a single owner thread or wavefront and sums in a
// fixed order (no atomics): results are bit-reproducible.
#include "common.h"
#include "fmm.h"
#include "sincos_cw.h"

#include <cmath>
#include <mutex>

namespace bem {

namespace {

constexpr double kInv16Pi2 = 0.0063325739776461107152;  // 1 / (16 pi^2)
enum { P0X = 0, P1X = 3, P2X = 6, NX = 9, AREA = 12, CX = 13 };

__device__ inline double2 mk(double a, double b) { return make_double2(a, b); }
__device__ inline float2 mk(float a, float b) { return make_float2(a, b); }
template <typename V>
__device__ inline V cmul(V a, V b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// conj(a) * b
template <typename V>
__device__ inline V cmulc(V a, V b) { return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
template <typename V>
__device__ inline V cadd(V a, V b) { return mk(a.x + b.x, a.y + b.y); }

template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

template <typename V> __device__ inline V from_d2(double2 v);
template <> __device__ inline double2 from_d2<double2>(double2 v) { return v; }
template <> __device__ inline float2 from_d2<float2>(double2 v) { return make_float2((float)v.x, (float)v.y); }

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------ setup ---
// A quadrilateral's row is the sum over its two integration triangles (qidx
// >= 0: geometry in hq, stride nh).
template <bool SINGLE>
__global__ void k_leaf_T(int64_t N, const double* __restrict__ g, const int64_t* __restrict__ qidx,
                         const double* __restrict__ hq, int64_t nh, const int64_t* __restrict__ ec,
                         const double* __restrict__ zc, const double* __restrict__ s, int nu,
                         const double2* __restrict__ cfac, double k, const double* __restrict__ ra,
                         const double* __restrict__ rb, const double* __restrict__ rw, int nq,
                         double2* __restrict__ T64, float2* __restrict__ T32) {
  const int64_t j = blockIdx.y;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nu) return;
  const int64_t idx = j * nu + v;
  const int64_t c = ec[j];
  const double sx = s[3 * v], sy = s[3 * v + 1], sz = s[3 * v + 2];
  const int64_t qj = qidx ? qidx[j] : -1;
  const int nrec = qj >= 0 ? 2 : 1;
  double sr = 0.0, si = 0.0;
  for (int h = 0; h < nrec; ++h) {
    const double* gg = qj >= 0 ? hq : g;
    const int64_t st = qj >= 0 ? nh : N, r = qj >= 0 ? 2 * qj + h : j;
    double P0[3], e1[3], e2[3];
    for (int d = 0; d < 3; ++d) {
      P0[d] = gg[(P0X + d) * st + r];
      e1[d] = gg[(P1X + d) * st + r] - P0[d];
      e2[d] = gg[(P2X + d) * st + r] - P0[d];
    }
    // exp(ik (z - y).s) = exp(ik (z - P0).s) exp(-ik (a e1 + b e2).s)
    const double base =
        k * ((zc[3 * c] - P0[0]) * sx + (zc[3 * c + 1] - P0[1]) * sy + (zc[3 * c + 2] - P0[2]) * sz);
    const double pe1 = k * (e1[0] * sx + e1[1] * sy + e1[2] * sz);
    const double pe2 = k * (e2[0] * sx + e2[1] * sy + e2[2] * sz);
    const double a2 = 2.0 * gg[AREA * st + r];
    if (SINGLE) {
      // rows of the complex-FP32 operator: phases in revolutions (the hardware
      // sine and cosine take revolutions), formed from FP64 per-row terms
      constexpr double kRev = 0.15915494309189533577;  // 1 / (2 pi)
      const float b0 = (float)(base * kRev), q1 = (float)(pe1 * kRev), q2 = (float)(pe2 * kRev);
      float ar = 0.0f, ai = 0.0f;
      for (int q = 0; q < nq; ++q) {
        const float ph = fmaf(-(float)rb[q], q2, fmaf(-(float)ra[q], q1, b0));
        const float w = (float)rw[q];
        ar = fmaf(w, __builtin_amdgcn_cosf(ph), ar);
        ai = fmaf(w, __builtin_amdgcn_sinf(ph), ai);
      }
      sr += (double)ar * a2;
      si += (double)ai * a2;
    } else {
      double ar = 0.0, ai = 0.0;
      for (int q = 0; q < nq; ++q) {
        double sn, cs;
        sincos_cw_lit(base - ra[q] * pe1 - rb[q] * pe2, &sn, &cs);
        ar += rw[q] * cs;
        ai += rw[q] * sn;
      }
      sr += ar * a2;
      si += ai * a2;
    }
  }
  if (SINGLE)
    T32[idx] = make_float2((float)sr, (float)si);
  else
    T64[idx] = make_double2(sr, si);
}

__global__ void k_leaf_S(int64_t N, const double* __restrict__ g, const int64_t* __restrict__ ec,
                         const double* __restrict__ zc, const double* __restrict__ s,
                         const double* __restrict__ w, int nu, double k, double gre, double gim,
                         double2* __restrict__ S64, float2* __restrict__ S32) {
  const int64_t i = blockIdx.y;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nu) return;
  const int64_t idx = i * nu + v;
  const int64_t c = ec[i];
  const double sx = s[3 * v], sy = s[3 * v + 1], sz = s[3 * v + 2];
  const double ph = k * ((g[CX * N + i] - zc[3 * c]) * sx + (g[(CX + 1) * N + i] - zc[3 * c + 1]) * sy +
                         (g[(CX + 2) * N + i] - zc[3 * c + 2]) * sz);
  double sn, cs;
  sincos(ph, &sn, &cs);
  const double sdn = sx * g[NX * N + i] + sy * g[(NX + 1) * N + i] + sz * g[(NX + 2) * N + i];
  // (1 - gamma ik s.n): gamma ik = -k gim + i k gre
  const double fr = 1.0 + k * gim * sdn, fi = -k * gre * sdn;
  // prefactor ik w / (16 pi^2)
  const double pre = k * w[v] * kInv16Pi2;
  // i pre (fr + i fi)(cs + i sn)
  const double ur = fr * cs - fi * sn, ui = fr * sn + fi * cs;
  const double r = -pre * ui, im = pre * ur;
  if (S64) S64[idx] = make_double2(r, im);
  if (S32) S32[idx] = make_float2((float)r, (float)im);
}

// Bonnet factors (2l+1)/(l+1) and l/(l+1), l < kLegMax (wavefront-uniform
// scalar loads in the node loop of k_translation)
constexpr int kLegMax = 128;
__constant__ double c_leg_a[kLegMax];
__constant__ double c_leg_b[kLegMax];

// one block per interaction pair; h_l by upward recurrence in shared memory
__global__ __launch_bounds__(256) void k_translation(int64_t npairs, const int64_t* __restrict__ pm,
                                                     const int64_t* __restrict__ pn,
                                                     const double* __restrict__ z,
                                                     const double* __restrict__ s, int nu, int L, double k,
                                                     double2* __restrict__ D64, float2* __restrict__ D32) {
  extern __shared__ double2 coef[];  // L + 1 values i^l (2l+1) h_l(k|X|)
  const int64_t q = blockIdx.x;
  if (q >= npairs) return;
  const int64_t a = pm[q], b = pn[q];
  const double X0 = z[3 * a] - z[3 * b], X1 = z[3 * a + 1] - z[3 * b + 1], X2 = z[3 * a + 2] - z[3 * b + 2];
  const double r = sqrt(X0 * X0 + X1 * X1 + X2 * X2);
  if (threadIdx.x == 0) {
    const double x = k * r;
    double sn, cs;
    sincos(x, &sn, &cs);
    double h0r = sn / x, h0i = -cs / x;
    double h1r = (sn - x * cs) / (x * x), h1i = -(cs + x * sn) / (x * x);
    for (int l = 0; l <= L; ++l) {
      double hr, hi;
      if (l == 0) { hr = h0r; hi = h0i; }
      else if (l == 1) { hr = h1r; hi = h1i; }
      else {
        const double f = (2.0 * (l - 1) + 1.0) / x;
        hr = f * h1r - h0r;
        hi = f * h1i - h0i;
        h0r = h1r; h0i = h1i;
        h1r = hr; h1i = hi;
      }
      // i^l
      double cr, ci;
      switch (l & 3) {
        case 0: cr = hr; ci = hi; break;
        case 1: cr = -hi; ci = hr; break;
        case 2: cr = -hr; ci = -hi; break;
        default: cr = hi; ci = -hr; break;
      }
      coef[l] = make_double2((2.0 * l + 1.0) * cr, (2.0 * l + 1.0) * ci);
    }
  }
  __syncthreads();
  const double u0 = X0 / r, u1 = X1 / r, u2 = X2 / r;
  for (int v = threadIdx.x; v < nu; v += blockDim.x) {
    const double ct = s[3 * v] * u0 + s[3 * v + 1] * u1 + s[3 * v + 2] * u2;
    double pm1 = 1.0, p = ct;
    double dr = coef[0].x, di = coef[0].y;
    if (L >= 1) {
      dr += coef[1].x * ct;
      di += coef[1].y * ct;
    }
    for (int l = 1; l < L; ++l) {
      // Bonnet: P_{l+1} = ((2l+1) x P_l - l P_{l-1}) / (l+1)
      const double pn1 = fma(c_leg_a[l] * ct, p, -c_leg_b[l] * pm1);
      pm1 = p;
      p = pn1;
      dr += coef[l + 1].x * p;
      di += coef[l + 1].y * p;
    }
    if (D64) D64[q * nu + v] = make_double2(dr, di);
    if (D32) D32[q * nu + v] = make_float2((float)dr, (float)di);
  }
}

__global__ void k_shift(int64_t nchild, const int64_t* __restrict__ parent, const double* __restrict__ zp,
                        const double* __restrict__ zc, const double* __restrict__ s, int nu, double k,
                        double2* __restrict__ S64, float2* __restrict__ S32) {
  const int64_t c = blockIdx.y;
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nu) return;
  const int64_t idx = c * nu + v;
  const int64_t p = parent[c];
  const double ph = k * ((zp[3 * p] - zc[3 * c]) * s[3 * v] + (zp[3 * p + 1] - zc[3 * c + 1]) * s[3 * v + 1] +
                         (zp[3 * p + 2] - zc[3 * c + 2]) * s[3 * v + 2]);
  double sn, cs;
  sincos(ph, &sn, &cs);
  if (S64) S64[idx] = make_double2(cs, sn);
  if (S32) S32[idx] = make_float2((float)cs, (float)sn);
}

// ------------------------------------------------------------ apply ---
// Source factor of the aggregation rows: c_j + ik s.n_j (the derivatives of
// H and E fold into the outgoing plane wave; Sec. 3.3.1).
template <typename T, typename V>
__device__ inline V source_factor(const FactorArgs& F, int64_t j, int v) {
  const T sx = (T)F.s[3 * v], sy = (T)F.s[3 * v + 1], sz = (T)F.s[3 * v + 2];
  const T sn = sx * (T)F.n[j] + sy * (T)F.n[F.N + j] + sz * (T)F.n[2 * F.N + j];
  T fr = 0, fi = (T)F.k * sn;
  if (F.cfac) {
    fr += (T)F.cfac[j].x;
    fi += (T)F.cfac[j].y;
  }
  return mk(fr, fi);
}

// The level-transfer kernels form a chain of short launches that runs beside
// the near-field kernel and the leaf translation; a raised wave priority lets
// their few instructions issue ahead of those long arithmetic and load streams.
__device__ inline void chain_priority() { __builtin_amdgcn_s_setprio(2); }

// sig_c(nu) = sum_{j in c} r_j(nu) x_j with r = Tm (CONJ: conj(Tm)) times the
// source factor when FACTOR
template <typename T, typename V, bool CONJ, bool FACTOR>
__global__ __launch_bounds__(256) void k_aggregate(const int64_t* __restrict__ ebeg,
                                                   const int64_t* __restrict__ eend, int nu,
                                                   const V* __restrict__ Tm, FactorArgs F,
                                                   const double2* __restrict__ x, V* __restrict__ sig) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (v >= nu) return;
  V acc = mk(T(0), T(0));
  // unrolled so that several rows are in flight per lane
#pragma unroll 8
  for (int64_t j = ebeg[c]; j < eend[c]; ++j) {
    V t = Tm[j * nu + v];
    if (CONJ) t = mk(t.x, -t.y);
    if (FACTOR) t = cmul(t, source_factor<T, V>(F, j, v));
    acc = cadd(acc, cmul(t, from_d2<V>(x[j])));
  }
  sig[c * nu + v] = acc;
}

__device__ inline double wsum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// y_i += sum_nu r_i(nu) loc_c(i)(nu) with r = Sm, or conj(Sm * factor) for
// the conjugate transpose of aggregation (CONJ; FACTOR adds the source factor)
template <typename T, typename V, bool CONJ, bool FACTOR>
__global__ __launch_bounds__(256) void k_disaggregate(int64_t N, const int64_t* __restrict__ ec, int nu,
                                                      const V* __restrict__ Sm, FactorArgs F,
                                                      const V* __restrict__ loc, double2* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= N) return;
  const int64_t c = ec[i];
  T ar = 0, ai = 0;
#pragma unroll 4
  for (int v = lane; v < nu; v += 64) {
    V a = Sm[i * nu + v];
    if (FACTOR) a = cmul(a, source_factor<T, V>(F, i, v));
    const V b = loc[c * nu + v];
    const T ay = CONJ ? -a.y : a.y;
    ar += a.x * b.x - ay * b.y;
    ai += a.x * b.y + ay * b.x;
  }
  const double sr = wsum((double)ar), si = wsum((double)ai);
  if (lane == 0) {
    double2 o = y[i];
    y[i] = make_double2(o.x + sr, o.y + si);
  }
}

// loc_m = sum_q D_(m, il[q]) sig_il[q] over m's entries q, with D_mn read from
// slot code[q] >> 1 at node v or, if code[q] & 1, at the antipodal node
// (t, j) -> (L-1-t, j+L mod 2L).  ADJ: loc_n = sum_q conj(D_(il[q], n)) sig_il[q]:
// the same slot with the flip inverted.
// ORDER 1 (slab): a one-dimensional grid whose blocks the hardware hands to
// the 8 XCDs in turn (block b to XCD b mod 8) is mapped so that XCD j serves
// the targets of the j-th eighth of the level in tree order: neighbouring
// targets share most of their interaction lists, so the source signatures
// they read stay in that XCD's L2.  ORDER 2 (node ranges): XCD j serves
// nodes [j nu / 8, (j + 1) nu / 8) of every target, in chunks of TPB, so its
// share of all the signatures (an eighth) fits its L2.
template <typename T, typename V, bool ADJ, int TPB, int ORDER>
__global__ __launch_bounds__(TPB) void k_translate(const int64_t* __restrict__ il_off,
                                                   const int64_t* __restrict__ il,
                                                   const int64_t* __restrict__ code, int L, int nu, int64_t nc,
                                                   const V* __restrict__ D, const V* __restrict__ sig,
                                                   V* __restrict__ loc) {
  int64_t m;
  int v;
  if (ORDER == 1) {
    const int nbx = (nu + TPB - 1) / TPB;
    const int64_t b = blockIdx.x;
    const int64_t xcd = b & 7, r = b >> 3;
    const int64_t m0 = nc * xcd / 8, m1 = nc * (xcd + 1) / 8;
    m = m0 + r / nbx;
    if (m >= m1) return;
    v = (int)(r % nbx) * TPB + threadIdx.x;
    if (v >= nu) return;
  } else if (ORDER == 2) {
    const int64_t b = blockIdx.x;
    const int xcd = (int)(b & 7);
    const int64_t r = b >> 3;
    const int n0 = (int)((int64_t)nu * xcd / 8), n1 = (int)((int64_t)nu * (xcd + 1) / 8);
    const int nch = ((nu + 7) / 8 + TPB - 1) / TPB;  // chunks per target and XCD (the widest range)
    m = r / nch;
    if (m >= nc) return;
    v = n0 + (int)(r % nch) * TPB + threadIdx.x;
    if (v >= n1) return;
  } else {
    m = blockIdx.y;
    v = blockIdx.x * TPB + threadIdx.x;
    if (v >= nu) return;
  }
  const int twoL = 2 * L;
  const int t = v / twoL, j = v - t * twoL;
  const int va = (L - 1 - t) * twoL + (j < L ? j + L : j - L);
  V acc = mk(T(0), T(0));
  const int64_t q0 = il_off[m], q1 = il_off[m + 1];
  int64_t q = q0;
  // four independent loads in flight per lane
  for (; q + 4 <= q1; q += 4) {
    V d[4], sg[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t c = code[q + u];
      const bool flip = ((c & 1) != 0) != ADJ;
      d[u] = D[(c >> 1) * nu + (flip ? va : v)];
      sg[u] = sig[il[q + u] * nu + v];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = cadd(acc, ADJ ? cmulc(d[u], sg[u]) : cmul(d[u], sg[u]));
  }
  for (; q < q1; ++q) {
    const int64_t c = code[q];
    const bool flip = ((c & 1) != 0) != ADJ;
    const V dv = D[(c >> 1) * nu + (flip ? va : v)];
    const V sv = sig[il[q] * nu + v];
    acc = cadd(acc, ADJ ? cmulc(dv, sv) : cmul(dv, sv));
  }
  loc[m * nu + v] = acc;
}

template <typename T, typename V>
__global__ __launch_bounds__(256) void k_up_equal(const int64_t* __restrict__ cbeg,
                                                  const int64_t* __restrict__ cend, int nu,
                                                  const V* __restrict__ shift, const V* __restrict__ sigc,
                                                  V* __restrict__ sigp) {
  chain_priority();
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t p = blockIdx.y;
  if (v >= nu) return;
  V acc = mk(T(0), T(0));
  for (int64_t c = cbeg[p]; c < cend[p]; ++c) acc = cadd(acc, cmul(shift[c * nu + v], sigc[c * nu + v]));
  sigp[p * nu + v] = acc;
}

template <typename T, typename V>
__global__ __launch_bounds__(256) void k_down_equal(const int64_t* __restrict__ parent, int nu,
                                                    const V* __restrict__ shift, const V* __restrict__ locp,
                                                    V* __restrict__ locc) {
  chain_priority();
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (v >= nu) return;
  const V add = cmulc(shift[c * nu + v], locp[parent[c] * nu + v]);
  locc[c * nu + v] = cadd(locc[c * nu + v], add);
}

// Level-transfer kernels: small dense products whose table (DFT matrix, or
// a cluster's input rows for the theta resampling) is shared by every row of
// a cluster.  A block holds kXferRows rows, one per wavefront, and stages
// the table in LDS when it fits in kXferTab bytes (TAB), so the table is
// read from L2 once per block instead of once per row.
constexpr int kXferRows = 4;
constexpr size_t kXferTab = 49152;
// row-blocked forms only for launches of at least this many blocks
constexpr int64_t kXferMinBlocks = 2048;

// out[c][t][mi] = sum_j val(j) Et[j][mi], Et stored j-major (consecutive lanes
// read consecutive mi).  mode 0: val(j) = in[c][t][j]; mode 1: val(j) =
// conj(shift[c][t][j]) in[parent[c]][t][j].
template <typename T, typename V, bool TAB>
__global__ __launch_bounds__(256) void k_dft(int nt, int nj, int nm, int rl, const V* __restrict__ in,
                                             const V* __restrict__ shift, const int64_t* __restrict__ parent,
                                             int mode, const V* __restrict__ Et, V* __restrict__ out) {
  chain_priority();
  extern __shared__ unsigned char xfer_smem[];
  V* row = reinterpret_cast<V*>(xfer_smem);  // kXferRows x rl (rl >= nj)
  V* tab = row + kXferRows * rl;             // nj x nm when TAB
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.x * kXferRows + w;
  const int64_t c = blockIdx.y;
  if (TAB)
    for (int i = threadIdx.x; i < nj * nm; i += 256) tab[i] = Et[i];
  if (t < nt) {
    const int64_t rowoff = (int64_t)t * nj;
    V* rw = row + w * rl;
    if (mode == 0) {
      const V* src = in + c * (int64_t)nt * nj + rowoff;
      for (int jj = lane; jj < nj; jj += 64) rw[jj] = src[jj];
    } else {
      const V* src = in + parent[c] * (int64_t)nt * nj + rowoff;
      const V* sh = shift + c * (int64_t)nt * nj + rowoff;
      for (int jj = lane; jj < nj; jj += 64) rw[jj] = cmulc(sh[jj], src[jj]);
    }
  }
  __syncthreads();
  if (t >= nt) return;  // no barrier below
  const V* E = TAB ? tab : Et;
  const V* rw = row + w * rl;
  V* o = out + (c * nt + t) * (int64_t)nm;
  for (int mi = lane; mi < nm; mi += 64) {
    V acc = mk(T(0), T(0));
    for (int jj = 0; jj < nj; ++jj) acc = cadd(acc, cmul(rw[jj], E[(int64_t)jj * nm + mi]));
    o[mi] = acc;
  }
}

// out[c][to][mi] = sum_ti M[to][ti][|m|] in[c][ti][mi], m = mi - mhalf; the
// cluster's input rows are the staged table.
template <typename T, typename V, bool TAB>
__global__ __launch_bounds__(256) void k_theta(int nto, int nti, int nm, int mhalf, int nmh, const T* __restrict__ M,
                                               const V* __restrict__ in, V* __restrict__ out) {
  chain_priority();
  extern __shared__ unsigned char xfer_smem[];
  V* tab = reinterpret_cast<V*>(xfer_smem);  // nti x nm when TAB
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int to = blockIdx.x * kXferRows + w;
  const int64_t c = blockIdx.y;
  const V* src = in + c * (int64_t)nti * nm;
  if (TAB) {
    for (int i = threadIdx.x; i < nti * nm; i += 256) tab[i] = src[i];
    __syncthreads();
  }
  if (to >= nto) return;  // no barrier below
  const V* S = TAB ? tab : src;
  const T* Mr = M + (int64_t)to * nti * nmh;
  V* o = out + (c * nto + to) * (int64_t)nm;
  for (int mi = lane; mi < nm; mi += 64) {
    int am = mi - mhalf;
    if (am < 0) am = -am;
    T ar = 0, ai = 0;
    for (int ti = 0; ti < nti; ++ti) {
      const V a = S[(int64_t)ti * nm + mi];
      const T wv = Mr[(int64_t)ti * nmh + am];
      ar += wv * a.x;
      ai += wv * a.y;
    }
    o[mi] = mk(ar, ai);
  }
}

// sigp[p][t][j] = sum_{c in children(p)} shift[c][t][j] sum_mi G[c][t][mi] E[mi][j];
// one wavefront per row t, lanes over j (up to 4 per lane, nj <= 256).
template <typename T, typename V, bool TAB>
__global__ __launch_bounds__(256) void k_up_idft(const int64_t* __restrict__ cbeg, const int64_t* __restrict__ cend,
                                                 int nt, int nj, int nm, int rl, const V* __restrict__ G,
                                                 const V* __restrict__ E, const V* __restrict__ shift,
                                                 V* __restrict__ sigp) {
  chain_priority();
  extern __shared__ unsigned char xfer_smem[];
  V* g = reinterpret_cast<V*>(xfer_smem);  // kXferRows x rl (rl >= nm)
  V* tab = g + kXferRows * rl;             // nm x nj when TAB
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.x * kXferRows + w;
  const bool act = t < nt;
  const int64_t p = blockIdx.y;
  if (TAB)
    for (int i = threadIdx.x; i < nm * nj; i += 256) tab[i] = E[i];
  const V* Et = TAB ? tab : E;
  V* gw = g + w * rl;
  V acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = mk(T(0), T(0));
  // every wavefront of the block walks the same children (uniform barriers)
  for (int64_t c = cbeg[p]; c < cend[p]; ++c) {
    __syncthreads();
    if (act) {
      const V* gc = G + (c * nt + t) * (int64_t)nm;
      for (int mi = lane; mi < nm; mi += 64) gw[mi] = gc[mi];
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int jj = lane + 64 * q;
        if (jj < nj) {
          V sacc = mk(T(0), T(0));
          for (int mi = 0; mi < nm; ++mi) sacc = cadd(sacc, cmul(gw[mi], Et[(int64_t)mi * nj + jj]));
          acc[q] = cadd(acc[q], cmul(shift[(c * nt + t) * (int64_t)nj + jj], sacc));
        }
      }
    }
  }
  if (act) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int jj = lane + 64 * q;
      if (jj < nj) sigp[(p * nt + t) * (int64_t)nj + jj] = acc[q];
    }
  }
}

// locc[c][t][j] += sum_mi K[c][t][mi] E[mi][j]; one wavefront per row t.
template <typename T, typename V, bool TAB>
__global__ __launch_bounds__(256) void k_down_idft(int nt, int nj, int nm, int rl, const V* __restrict__ K,
                                                   const V* __restrict__ E, V* __restrict__ locc) {
  chain_priority();
  extern __shared__ unsigned char xfer_smem[];
  V* kk = reinterpret_cast<V*>(xfer_smem);  // kXferRows x rl (rl >= nm)
  V* tab = kk + kXferRows * rl;             // nm x nj when TAB
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int t = blockIdx.x * kXferRows + w;
  const int64_t c = blockIdx.y;
  if (TAB)
    for (int i = threadIdx.x; i < nm * nj; i += 256) tab[i] = E[i];
  V* kw = kk + w * rl;
  if (t < nt) {
    const V* kr = K + (c * nt + t) * (int64_t)nm;
    for (int mi = lane; mi < nm; mi += 64) kw[mi] = kr[mi];
  }
  __syncthreads();
  if (t >= nt) return;  // no barrier below
  const V* Et = TAB ? tab : E;
  for (int jj = lane; jj < nj; jj += 64) {
    V sacc = mk(T(0), T(0));
    for (int mi = 0; mi < nm; ++mi) sacc = cadd(sacc, cmul(kw[mi], Et[(int64_t)mi * nj + jj]));
    const int64_t o = (c * nt + t) * (int64_t)nj + jj;
    locc[o] = cadd(locc[o], sacc);
  }
}

// One-row-per-block forms (table read from L2), used where a level has too
// few clusters for the row-blocked forms to fill the chip.
// One 64-lane block per (cluster c, row t): out[c][t][mi] = sum_j val(j) Et[j][mi]
// with Et the DFT table stored j-major (consecutive lanes read consecutive mi).
// mode 0: val(j) = in[c][t][j]; mode 1: val(j) = conj(shift[c][t][j]) in[parent[c]][t][j].
template <typename T, typename V>
__global__ __launch_bounds__(64) void k_dft_row(int nt, int nj, int nm, const V* __restrict__ in,
                                            const V* __restrict__ shift, const int64_t* __restrict__ parent,
                                            int mode, const V* __restrict__ Et, V* __restrict__ out) {
  chain_priority();
  __shared__ V row[256];
  const int t = blockIdx.x;
  const int64_t c = blockIdx.y;
  const int64_t rowoff = (int64_t)t * nj;
  if (mode == 0) {
    const V* src = in + c * (int64_t)nt * nj + rowoff;
    for (int j = threadIdx.x; j < nj; j += 64) row[j] = src[j];
  } else {
    const V* src = in + parent[c] * (int64_t)nt * nj + rowoff;
    const V* sh = shift + c * (int64_t)nt * nj + rowoff;
    for (int j = threadIdx.x; j < nj; j += 64) row[j] = cmulc(sh[j], src[j]);
  }
  __syncthreads();
  V* o = out + (c * nt + t) * (int64_t)nm;
  for (int mi = threadIdx.x; mi < nm; mi += 64) {
    V acc = mk(T(0), T(0));
    for (int j = 0; j < nj; ++j) acc = cadd(acc, cmul(row[j], Et[(int64_t)j * nm + mi]));
    o[mi] = acc;
  }
}

// One block per (parent p, row t), lanes over j:
// sigp[p][t][j] = sum_{c in children(p)} shift[c][t][j] sum_mi G[c][t][mi] E[mi][j]
template <typename T, typename V>
__global__ __launch_bounds__(128) void k_up_idft_row(const int64_t* __restrict__ cbeg, const int64_t* __restrict__ cend,
                                                 int nt, int nj, int nm, const V* __restrict__ G,
                                                 const V* __restrict__ E, const V* __restrict__ shift,
                                                 V* __restrict__ sigp) {
  chain_priority();
  __shared__ V g[256];
  const int t = blockIdx.x;
  const int64_t p = blockIdx.y;
  V acc[2] = {mk(T(0), T(0)), mk(T(0), T(0))};
  for (int64_t c = cbeg[p]; c < cend[p]; ++c) {
    __syncthreads();
    const V* gc = G + (c * nt + t) * (int64_t)nm;
    for (int mi = threadIdx.x; mi < nm; mi += blockDim.x) g[mi] = gc[mi];
    __syncthreads();
    for (int r = 0; r < 2; ++r) {
      const int j = threadIdx.x + r * blockDim.x;
      if (j >= nj) continue;
      V s = mk(T(0), T(0));
      for (int mi = 0; mi < nm; ++mi) s = cadd(s, cmul(g[mi], E[(int64_t)mi * nj + j]));
      acc[r] = cadd(acc[r], cmul(shift[(c * nt + t) * (int64_t)nj + j], s));
    }
  }
  for (int r = 0; r < 2; ++r) {
    const int j = threadIdx.x + r * blockDim.x;
    if (j < nj) sigp[(p * nt + t) * (int64_t)nj + j] = acc[r];
  }
}

// One block per (cluster c, row t), lanes over j: locc[c][t][j] += sum_mi K[c][t][mi] E[mi][j]
template <typename T, typename V>
__global__ __launch_bounds__(128) void k_down_idft_row(int nt, int nj, int nm, const V* __restrict__ K,
                                                   const V* __restrict__ E, V* __restrict__ locc) {
  chain_priority();
  __shared__ V kk[256];
  const int t = blockIdx.x;
  const int64_t c = blockIdx.y;
  const V* kr = K + (c * nt + t) * (int64_t)nm;
  for (int mi = threadIdx.x; mi < nm; mi += blockDim.x) kk[mi] = kr[mi];
  __syncthreads();
  for (int j = threadIdx.x; j < nj; j += blockDim.x) {
    V s = mk(T(0), T(0));
    for (int mi = 0; mi < nm; ++mi) s = cadd(s, cmul(kk[mi], E[(int64_t)mi * nj + j]));
    const int64_t o = (c * nt + t) * (int64_t)nj + j;
    locc[o] = cadd(locc[o], s);
  }
}

// ---- level transfer on the matrix cores ------------------------------------
// The azimuthal DFTs of the resampling are products of a level's rows (R =
// clusters x theta rows, K complex values each) with one K x N complex table
// shared by all rows.  Written on interleaved reals, the complex product is
// one real product: row (2K reals) times the 2K x 2N table
//   B'[2k + a][2n + b] = Re B[k][n] (a = b),  Im B[k][n] (a = 0, b = 1),  -Im B[k][n] (a = 1, b = 0),
// whose interleaved output is the complex result.  One wavefront computes a
// 16-row x 16-real-column tile with 16 x 16 x 4 MFMA steps
// (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64): operand A[i][k] in lane
// i + 16k, B[k][j] in lane j + 16k; result D[i][j] in lane j + 16 (i / 4),
// element i % 4 (FP32) and in lane j + 16 (i % 4), element i / 4 (FP64).
// Consecutive wavefronts take the column tiles of one row tile, so the rows
// are read from L2 once per block; the table (a few tens of KB) stays in L2.
// Used where the table is too large for the LDS-staged VALU form (the
// row-per-block VALU fallback then reads it from L2 per row): measured alone
// at c2, FP64 upward DFT 152 x 34 rows (K = 68, N = 67) 27.1 -> 16.4 us and
// downward inverse DFT (K = 67, N = 68) 26.2 -> 19.5 us; where the table
// fits LDS the VALU forms are as fast or faster (these products are bound
// by memory latency, not arithmetic), and the shifted-parent form (conj(shift)
// times the parent row, formed per operand) lost everywhere.
typedef float mf_f4 __attribute__((ext_vector_type(4)));
typedef double mf_d4 __attribute__((ext_vector_type(4)));
template <typename T> struct Mfma;
template <> struct Mfma<float> {
  using acc = mf_f4;
  __device__ static acc op(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int lq, int v) { return 4 * lq + v; }  // row of result element v in lane group lq
};
template <> struct Mfma<double> {
  using acc = mf_d4;
  __device__ static acc op(double a, double b, acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int lq, int v) { return lq + 4 * v; }
};

constexpr int kMfmaWaves = 4;  // wavefronts per block

// ACC false: out[r][0..N) = in[r][0..K) B;  ACC true: out[r][n] += (in[r] B)[n].
// The K steps run in chunks of CH whose operands are loaded together.
template <typename T, typename V, bool ACC, int CH>
__global__ __launch_bounds__(64 * kMfmaWaves) void k_xfer_mfma(int64_t R, int K, int N, const V* __restrict__ in,
                                                              const V* __restrict__ B, V* __restrict__ out) {
  chain_priority();
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int K2 = 2 * K, N2 = 2 * N;
  const int nut = (N2 + 15) >> 4;
  const int64_t g = (int64_t)blockIdx.x * kMfmaWaves + (threadIdx.x >> 6);
  const int64_t row0 = (g / nut) * 16;
  const int u = (int)(g % nut);
  if (row0 >= R) return;  // wavefront-uniform
  const int ks = (K2 + 3) >> 2;
  const int64_t r = row0 + li;
  const bool rok = r < R;
  const T* src = reinterpret_cast<const T*>(in);
  const int nn = 16 * u + li;  // this lane's B' column and result column
  const bool nok = nn < N2;
  const int n = nn >> 1, bpart = nn & 1;
  const T* Bs = reinterpret_cast<const T*>(B);
  typename Mfma<T>::acc acc = {T(0), T(0), T(0), T(0)};
  for (int s0 = 0; s0 < ks; s0 += CH) {
    T a[CH], b[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      a[q] = T(0);
      b[q] = T(0);
      const int kk = 4 * (s0 + q) + lq;
      if (kk < K2) {
        if (rok) a[q] = src[r * K2 + kk];
        if (nok) {
          const int apart = kk & 1;
          const T e = Bs[2 * ((kk >> 1) * N + n) + (apart != bpart)];
          b[q] = (apart && !bpart) ? -e : e;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (s0 + q < ks) acc = Mfma<T>::op(a[q], b[q], acc);  // uniform condition
  }
  if (nok) {
    T* o = reinterpret_cast<T*>(out);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t rr = row0 + Mfma<T>::row(lq, v);
      if (rr < R) {
        if (ACC)
          o[rr * N2 + nn] += acc[v];
        else
          o[rr * N2 + nn] = acc[v];
      }
    }
  }
}

// Host side: the matrix-core form of a rows-times-table transfer product.
template <typename T, typename V, bool ACC>
void xfer_mfma(int64_t R, int K, int N, const V* in, const V* B, V* out, hipStream_t st) {
  const int64_t waves = ((R + 15) / 16) * ((2 * N + 15) / 16);
  const dim3 grid((unsigned)((waves + kMfmaWaves - 1) / kMfmaWaves));
  hipLaunchKernelGGL((k_xfer_mfma<T, V, ACC, 16>), grid, dim3(64 * kMfmaWaves), 0, st, R, K, N, in, B, out);
}

}  // namespace

// ------------------------------------------------------------ launchers ---
// The Bonnet factors do not depend on the problem: uploaded once per device,
// flag and upload under one lock (meshes may be set up from several threads).
void ensure_legendre_factors() {
  static std::mutex mu;
  static bool leg_ready[64] = {};
  int dev = 0;
  BEM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error(BEM_E_HIP, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!leg_ready[dev]) {
    double a[kLegMax], b[kLegMax];
    for (int l = 0; l < kLegMax; ++l) {
      a[l] = (2.0 * l + 1.0) / (l + 1.0);
      b[l] = (double)l / (l + 1.0);
    }
    BEM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_leg_a), a, sizeof(a)));
    BEM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_leg_b), b, sizeof(b)));
    leg_ready[dev] = true;
  }
}
void launch_fmm_leaf_T(int64_t N, const double* geom, const int64_t* qidx, const double* hq, int64_t nh,
                       const int64_t* ec, const double* zc, const double* s, int nu, const double2* cfac, double k,
                       const double* ra, const double* rb, const double* rw, int nq, double2* T64, float2* T32,
                       hipStream_t st) {
  if (N <= 0 || nu <= 0) return;
  if (nh == 0) qidx = nullptr;
  if (T64)
    hipLaunchKernelGGL(k_leaf_T<false>, dim3(nblk(nu, 256), (unsigned)N), dim3(256), 0, st, N, geom, qidx, hq, nh,
                       ec, zc, s, nu, cfac, k, ra, rb, rw, nq, T64, nullptr);
  if (T32)
    hipLaunchKernelGGL(k_leaf_T<true>, dim3(nblk(nu, 256), (unsigned)N), dim3(256), 0, st, N, geom, qidx, hq, nh,
                       ec, zc, s, nu, cfac, k, ra, rb, rw, nq, nullptr, T32);
}

void launch_fmm_leaf_S(int64_t N, const double* geom, const int64_t* ec, const double* zc, const double* s,
                       const double* w, int nu, double k, double gre, double gim, double2* S64, float2* S32,
                       hipStream_t st) {
  if (N <= 0 || nu <= 0) return;
  hipLaunchKernelGGL(k_leaf_S, dim3(nblk(nu, 256), (unsigned)N), dim3(256), 0, st, N, geom, ec, zc, s, w, nu, k, gre, gim,
                     S64, S32);
}

void launch_fmm_translation(int64_t npairs, const int64_t* pm, const int64_t* pn, const double* z,
                            const double* s, int nu, int L, double k, double2* D64, float2* D32,
                            hipStream_t st) {
  if (npairs <= 0) return;
  ensure_legendre_factors();
  hipLaunchKernelGGL(k_translation, dim3((unsigned)npairs), dim3(256), (L + 1) * sizeof(double2), st, npairs, pm, pn, z, s,
                     nu, L, k, D64, D32);
}

void launch_fmm_shift(int64_t nchild, const int64_t* parent, const double* zp, const double* zc,
                      const double* s, int nu, double k, double2* S64, float2* S32, hipStream_t st) {
  if (nchild <= 0 || nu <= 0) return;
  hipLaunchKernelGGL(k_shift, dim3(nblk(nu, 256), (unsigned)nchild), dim3(256), 0, st, nchild, parent, zp, zc, s, nu, k, S64,
                     S32);
}

template <typename T, typename V>
void launch_fmm_aggregate(int64_t nclust, const int64_t* ebeg, const int64_t* eend, int nu, const V* Tm,
                          const FactorArgs* F, const double2* x, V* sig, bool conj_rows, hipStream_t st) {
  if (nclust <= 0) return;
  const dim3 grid(nblk(nu, 256), (unsigned)nclust);
  FactorArgs fa = F ? *F : FactorArgs{};
  if (conj_rows) {
    if (F) hipLaunchKernelGGL((k_aggregate<T, V, true, true>), grid, dim3(256), 0, st, ebeg, eend, nu, Tm, fa, x, sig);
    else hipLaunchKernelGGL((k_aggregate<T, V, true, false>), grid, dim3(256), 0, st, ebeg, eend, nu, Tm, fa, x, sig);
  } else {
    if (F) hipLaunchKernelGGL((k_aggregate<T, V, false, true>), grid, dim3(256), 0, st, ebeg, eend, nu, Tm, fa, x, sig);
    else hipLaunchKernelGGL((k_aggregate<T, V, false, false>), grid, dim3(256), 0, st, ebeg, eend, nu, Tm, fa, x, sig);
  }
}

template <typename T, typename V>
void launch_fmm_disaggregate(int64_t N, const int64_t* ec, int nu, const V* Sm, const FactorArgs* F, const V* loc,
                             double2* y, bool conj_rows, hipStream_t st) {
  if (N <= 0) return;
  FactorArgs fa = F ? *F : FactorArgs{};
  const dim3 grid(nblk(N, 4));
  if (conj_rows) {
    if (F) hipLaunchKernelGGL((k_disaggregate<T, V, true, true>), grid, dim3(256), 0, st, N, ec, nu, Sm, fa, loc, y);
    else hipLaunchKernelGGL((k_disaggregate<T, V, true, false>), grid, dim3(256), 0, st, N, ec, nu, Sm, fa, loc, y);
  } else {
    if (F) hipLaunchKernelGGL((k_disaggregate<T, V, false, true>), grid, dim3(256), 0, st, N, ec, nu, Sm, fa, loc, y);
    else hipLaunchKernelGGL((k_disaggregate<T, V, false, false>), grid, dim3(256), 0, st, N, ec, nu, Sm, fa, loc, y);
  }
}

template <typename T, typename V, int TPB, int ORDER>
void translate_shape(int64_t nc, const int64_t* il_off, const int64_t* il, const int64_t* code, bool adjoint, int L,
                     int nu, const V* D, const V* sig, V* loc, hipStream_t st) {
  dim3 grid(nblk(nu, TPB), (unsigned)nc);
  if (ORDER == 1) grid = dim3((unsigned)(8 * ((nc + 7) / 8) * nblk(nu, TPB)));
  if (ORDER == 2) grid = dim3((unsigned)(8 * nc * nblk((nu + 7) / 8, TPB)));
  if (adjoint)
    hipLaunchKernelGGL((k_translate<T, V, true, TPB, ORDER>), grid, dim3(TPB), 0, st, il_off, il, code, L, nu, nc, D,
                       sig, loc);
  else
    hipLaunchKernelGGL((k_translate<T, V, false, TPB, ORDER>), grid, dim3(TPB), 0, st, il_off, il, code, L, nu, nc,
                       D, sig, loc);
}

template <typename T, typename V, int TPB>
void translate_tpb(int64_t nc, const int64_t* il_off, const int64_t* il, const int64_t* code, bool adjoint, int L,
                   int nu, const V* D, const V* sig, V* loc, int order, hipStream_t st) {
  if (order == 1) translate_shape<T, V, TPB, 1>(nc, il_off, il, code, adjoint, L, nu, D, sig, loc, st);
  else if (order == 2) translate_shape<T, V, TPB, 2>(nc, il_off, il, code, adjoint, L, nu, D, sig, loc, st);
  else translate_shape<T, V, TPB, 0>(nc, il_off, il, code, adjoint, L, nu, D, sig, loc, st);
}

// tpb: 64, 128 or 256 threads per block; + kTranslateSlab: the XCD slab
// order, + kTranslateNodes: the XCD node-range order
template <typename T, typename V>
void launch_fmm_translate(int64_t nc, const int64_t* il_off, const int64_t* il, const int64_t* code, bool adjoint,
                          int L, int nu, const V* D, const V* sig, V* loc, int tpb, hipStream_t st) {
  if (nc <= 0) return;
  const int order = (tpb & kTranslateSlab) ? 1 : (tpb & kTranslateNodes) ? 2 : 0;
  tpb &= ~kTranslateFlags;
  if (tpb == 128) translate_tpb<T, V, 128>(nc, il_off, il, code, adjoint, L, nu, D, sig, loc, order, st);
  else if (tpb == 256) translate_tpb<T, V, 256>(nc, il_off, il, code, adjoint, L, nu, D, sig, loc, order, st);
  else translate_tpb<T, V, 64>(nc, il_off, il, code, adjoint, L, nu, D, sig, loc, order, st);
}

template <typename T, typename V>
void launch_fmm_up_equal(int64_t np, const int64_t* cbeg, const int64_t* cend, int nu, const V* shift,
                         const V* sigc, V* sigp, hipStream_t st) {
  if (np <= 0) return;
  hipLaunchKernelGGL((k_up_equal<T, V>), dim3(nblk(nu, 256), (unsigned)np), dim3(256), 0, st, cbeg, cend, nu,
                     shift, sigc, sigp);
}

template <typename T, typename V>
void launch_fmm_down_equal(int64_t nchild, const int64_t* parent, int nu, const V* shift, const V* locp,
                           V* locc, hipStream_t st) {
  if (nchild <= 0) return;
  hipLaunchKernelGGL((k_down_equal<T, V>), dim3(nblk(nu, 256), (unsigned)nchild), dim3(256), 0, st, parent, nu,
                     shift, locp, locc);
}

template <typename T, typename V>
void launch_fmm_dft(int64_t nc, int nt, int nj, int nm, const V* in, const V* shift, const int64_t* parent,
                    int mode, const V* Et, V* out, hipStream_t st) {
  if (nc <= 0 || nt <= 0) return;
  const dim3 grid((unsigned)((nt + kXferRows - 1) / kXferRows), (unsigned)nc);
  const int rl = (nj + 1) & ~1;
  const size_t rows = kXferRows * (size_t)rl * sizeof(V), tab = (size_t)nj * nm * sizeof(V);
  if (mode == 0 && tab > kXferTab) {  // matrix cores where the table cannot be staged
    xfer_mfma<T, V, false>(nc * nt, nj, nm, in, Et, out, st);
    return;
  }
  if (tab <= kXferTab && (int64_t)grid.x * nc >= kXferMinBlocks)
    hipLaunchKernelGGL((k_dft<T, V, true>), grid, dim3(256), rows + tab, st, nt, nj, nm, rl, in, shift, parent, mode,
                       Et, out);
  else
    hipLaunchKernelGGL((k_dft_row<T, V>), dim3((unsigned)nt, (unsigned)nc), dim3(64), 0, st, nt, nj, nm, in, shift,
                       parent, mode, Et, out);
}

template <typename T, typename V>
void launch_fmm_theta(int64_t nc, int nto, int nti, int nm, int mhalf, const T* M, const V* in, V* out,
                      hipStream_t st) {
  if (nc <= 0 || nto <= 0) return;
  const dim3 grid((unsigned)((nto + kXferRows - 1) / kXferRows), (unsigned)nc);
  const size_t tab = (size_t)nti * nm * sizeof(V);
  if (tab <= kXferTab)
    hipLaunchKernelGGL((k_theta<T, V, true>), grid, dim3(256), tab, st, nto, nti, nm, mhalf, mhalf + 1, M, in, out);
  else
    hipLaunchKernelGGL((k_theta<T, V, false>), grid, dim3(256), 0, st, nto, nti, nm, mhalf, mhalf + 1, M, in, out);
}

template <typename T, typename V>
void launch_fmm_up_idft(int64_t np, const int64_t* cbeg, const int64_t* cend, int nt, int nj, int nm,
                        const V* G, const V* E, const V* shift, V* sigp, hipStream_t st) {
  if (np <= 0 || nt <= 0) return;
  const dim3 grid((unsigned)((nt + kXferRows - 1) / kXferRows), (unsigned)np);
  const int rl = (nm + 1) & ~1;
  const size_t rows = kXferRows * (size_t)rl * sizeof(V), tab = (size_t)nm * nj * sizeof(V);
  if (tab <= kXferTab) {  // each block also walks the children: few blocks suffice
    hipLaunchKernelGGL((k_up_idft<T, V, true>), grid, dim3(256), rows + tab, st, cbeg, cend, nt, nj, nm, rl, G, E,
                       shift, sigp);
  } else {
    // one wavefront covers nj <= 64; the kernel walks two chunks of blockDim
    const unsigned threads = nj <= 64 ? 64 : 128;
    hipLaunchKernelGGL((k_up_idft_row<T, V>), dim3((unsigned)nt, (unsigned)np), dim3(threads), 0, st, cbeg, cend, nt,
                       nj, nm, G, E, shift, sigp);
  }
}

template <typename T, typename V>
void launch_fmm_down_idft(int64_t nc, int nt, int nj, int nm, const V* K, const V* E, V* locc,
                          hipStream_t st) {
  if (nc <= 0 || nt <= 0) return;
  const dim3 grid((unsigned)((nt + kXferRows - 1) / kXferRows), (unsigned)nc);
  const int rl = (nm + 1) & ~1;
  const size_t rows = kXferRows * (size_t)rl * sizeof(V), tab = (size_t)nm * nj * sizeof(V);
  if (tab > kXferTab) {  // matrix cores where the table cannot be staged
    xfer_mfma<T, V, true>(nc * nt, nm, nj, K, E, locc, st);
    return;
  }
  if (tab <= kXferTab && (int64_t)grid.x * nc >= kXferMinBlocks) {
    hipLaunchKernelGGL((k_down_idft<T, V, true>), grid, dim3(256), rows + tab, st, nt, nj, nm, rl, K, E, locc);
  } else {
    const unsigned threads = nj <= 64 ? 64 : 128;
    hipLaunchKernelGGL((k_down_idft_row<T, V>), dim3((unsigned)nt, (unsigned)nc), dim3(threads), 0, st, nt, nj, nm, K,
                       E, locc);
  }
}

#define BEM_FMM_INST(T, V)                                                                                    \
  template void launch_fmm_aggregate<T, V>(int64_t, const int64_t*, const int64_t*, int, const V*,            \
                                           const FactorArgs*, const double2*, V*, bool, hipStream_t);         \
  template void launch_fmm_disaggregate<T, V>(int64_t, const int64_t*, int, const V*, const FactorArgs*,      \
                                              const V*, double2*, bool, hipStream_t);                         \
  template void launch_fmm_translate<T, V>(int64_t, const int64_t*, const int64_t*, const int64_t*, bool, int, \
                                           int, const V*, const V*, V*, int, hipStream_t);                    \
  template void launch_fmm_up_equal<T, V>(int64_t, const int64_t*, const int64_t*, int, const V*, const V*,   \
                                          V*, hipStream_t);                                                   \
  template void launch_fmm_down_equal<T, V>(int64_t, const int64_t*, int, const V*, const V*, V*,             \
                                            hipStream_t);                                                     \
  template void launch_fmm_dft<T, V>(int64_t, int, int, int, const V*, const V*, const int64_t*, int,         \
                                     const V*, V*, hipStream_t);                                              \
  template void launch_fmm_theta<T, V>(int64_t, int, int, int, int, const T*, const V*, V*, hipStream_t);     \
  template void launch_fmm_up_idft<T, V>(int64_t, const int64_t*, const int64_t*, int, int, int, const V*,    \
                                         const V*, const V*, V*, hipStream_t);                                \
  template void launch_fmm_down_idft<T, V>(int64_t, int, int, int, const V*, const V*, V*, hipStream_t);

BEM_FMM_INST(double, double2)
BEM_FMM_INST(float, float2)

namespace {

// coefficients of the translation operator per (point cluster, leaf cluster)
// pair; h_l by upward recurrence in FP64 (as k_translation)
__global__ void k_grid_coef(int64_t npairs, const int64_t* __restrict__ pair_p, const int64_t* __restrict__ pair_c,
                            const double* __restrict__ zp, const double* __restrict__ zc, double k, int L,
                            double2* __restrict__ coef, double* __restrict__ dir) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= npairs) return;
  const int64_t a = pair_p[q], b = pair_c[q];
  const double X0 = zp[3 * a] - zc[3 * b], X1 = zp[3 * a + 1] - zc[3 * b + 1], X2 = zp[3 * a + 2] - zc[3 * b + 2];
  const double r = sqrt(X0 * X0 + X1 * X1 + X2 * X2);
  dir[3 * q] = X0 / r;
  dir[3 * q + 1] = X1 / r;
  dir[3 * q + 2] = X2 / r;
  const double x = k * r;
  double sn, cs;
  sincos(x, &sn, &cs);
  double h0r = sn / x, h0i = -cs / x;
  double h1r = (sn - x * cs) / (x * x), h1i = -(cs + x * sn) / (x * x);
  double2* c = coef + q * (int64_t)(L + 1);
  for (int l = 0; l <= L; ++l) {
    double hr, hi;
    if (l == 0) {
      hr = h0r;
      hi = h0i;
    } else if (l == 1) {
      hr = h1r;
      hi = h1i;
    } else {
      const double f = (2.0 * (l - 1) + 1.0) / x;
      hr = f * h1r - h0r;
      hi = f * h1i - h0i;
      h0r = h1r;
      h0i = h1i;
      h1r = hr;
      h1i = hi;
    }
    double cr, ci;  // i^l h_l
    switch (l & 3) {
      case 0: cr = hr; ci = hi; break;
      case 1: cr = -hi; ci = hr; break;
      case 2: cr = -hr; ci = -hi; break;
      default: cr = hi; ci = -hr; break;
    }
    c[l] = make_double2((2.0 * l + 1.0) * cr, (2.0 * l + 1.0) * ci);
  }
}

// one block per point cluster, threads over the sphere nodes; the far pairs
// of the cluster in a fixed order (deterministic), the translation values
// from the Legendre series (Bonnet recurrence) on the fly
__global__ __launch_bounds__(256) void k_grid_translate(const int64_t* __restrict__ far_off,
                                                        const int64_t* __restrict__ pair_c,
                                                        const double2* __restrict__ coef,
                                                        const double* __restrict__ dir, int L, int nu,
                                                        const double* __restrict__ s,
                                                        const double2* __restrict__ sigA,
                                                        const double2* __restrict__ sigB,
                                                        double2* __restrict__ loc) {
  const int64_t P = blockIdx.x;
  const int64_t q0 = far_off[P], q1 = far_off[P + 1];
  for (int v = threadIdx.x; v < nu; v += blockDim.x) {
    const double sx = s[3 * v], sy = s[3 * v + 1], sz = s[3 * v + 2];
    double ar = 0.0, ai = 0.0;
    for (int64_t q = q0; q < q1; ++q) {
      const double mu = sx * dir[3 * q] + sy * dir[3 * q + 1] + sz * dir[3 * q + 2];
      const double2* c = coef + q * (int64_t)(L + 1);
      double pm1 = 1.0, p = mu;
      double dr = c[0].x, di = c[0].y;
      if (L >= 1) {
        dr = fma(c[1].x, mu, dr);
        di = fma(c[1].y, mu, di);
      }
      for (int l = 1; l < L; ++l) {
        const double pn = fma(c_leg_a[l] * mu, p, -c_leg_b[l] * pm1);
        pm1 = p;
        p = pn;
        dr = fma(c[l + 1].x, p, dr);
        di = fma(c[l + 1].y, p, di);
      }
      const int64_t cidx = pair_c[q] * nu + v;
      const double2 a = sigA[cidx], b = sigB[cidx];
      const double gr = a.x + b.x, gi = a.y + b.y;
      ar += dr * gr - di * gi;
      ai += dr * gi + di * gr;
    }
    loc[P * nu + v] = make_double2(ar, ai);
  }
}

}  // namespace

void launch_grid_coef(int64_t npairs, const int64_t* pair_p, const int64_t* pair_c, const double* zp,
                      const double* zc, double k, int L, double2* coef, double* dir, hipStream_t st) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(k_grid_coef, dim3(nblk(npairs, 128)), dim3(128), 0, st, npairs, pair_p, pair_c, zp, zc, k, L,
                     coef, dir);
}

void launch_grid_translate(int64_t npc, const int64_t* far_off, const int64_t* pair_c, const double2* coef,
                           const double* dir, int L, int nu, const double* s, const double2* sigA,
                           const double2* sigB, double2* loc, hipStream_t st) {
  if (npc <= 0) return;
  ensure_legendre_factors();
  hipLaunchKernelGGL(k_grid_translate, dim3((unsigned)npc), dim3(256), 0, st, far_off, pair_c, coef, dir, L, nu, s,
                     sigA, sigB, loc);
}

}  // namespace bem
