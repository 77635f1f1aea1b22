// Device launchers of the multilevel FMM far field (fmm.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bem {

// Source factor c_j + ik s.n_j applied on the fly to the leaf aggregation rows.
struct FactorArgs {
  int64_t N;
  const double* s;       // leaf sphere nodes (3 per node)
  const double* n;       // element normals, field-major: n[d * N + j] (tree order)
  const double2* cfac;   // c_j (NULL: sound-hard)
  double k;
};

// ---------------------------------------------------------------- setup ---
// Outputs of the setup kernels are written in FP64 and/or FP32 (a NULL
// pointer skips that copy).
// Leaf aggregation rows T[j][nu] = int_Gj exp(ik (z_c(j) - y).s) dy (the source
// factor is applied when the rows are used)
// (conical rule with nq points: rule_a, rule_b, rule_w in device memory; a
// quadrilateral, qidx[j] >= 0, integrated over its two halves in hq, stride nh).
void launch_fmm_leaf_T(int64_t N, const double* geom, const int64_t* qidx, const double* hq, int64_t nh,
                       const int64_t* elem_cluster, const double* zc, const double* s, int nu, const double2* cfac,
                       double k, const double* ra, const double* rb, const double* rw, int nq, double2* T64,
                       float2* T32, hipStream_t st);
// Leaf disaggregation rows S'[i][nu] = ik/(16 pi^2) w_nu (1 - gamma ik s.n_i) exp(ik (x_i - z).s)
void launch_fmm_leaf_S(int64_t N, const double* geom, const int64_t* elem_cluster, const double* zc,
                       const double* s, const double* w, int nu, double k, double gre, double gim,
                       double2* S64, float2* S32, hipStream_t st);
// Translation values D[pair][nu] = sum_{l<=L} i^l (2l+1) h_l(k|X|) P_l(Xh.s), X = z_m - z_n
void launch_fmm_translation(int64_t npairs, const int64_t* pair_m, const int64_t* pair_n, const double* z,
                            const double* s, int nu, int L, double k, double2* D64, float2* D32,
                            hipStream_t st);
// Shift phases exp(ik (z_parent - z_child).s) on the parent grid, per child.
void launch_fmm_shift(int64_t nchild, const int64_t* parent, const double* zp, const double* zc,
                      const double* s, int nu, double k, double2* S64, float2* S32, hipStream_t st);

// ---------------------------------------------------------------- apply ---
// T = double (V = double2) or float (V = float2)
// conj_rows: use the complex conjugate of the row matrix (adjoint passes);
// F: multiply the rows by the source factor (NULL: plain rows)
template <typename T, typename V>
void launch_fmm_aggregate(int64_t nclust, const int64_t* ebeg, const int64_t* eend, int nu, const V* Tm,
                          const FactorArgs* F, const double2* x, V* sig, bool conj_rows, hipStream_t st);
template <typename T, typename V>
void launch_fmm_disaggregate(int64_t N, const int64_t* elem_cluster, int nu, const V* Sm, const FactorArgs* F,
                             const V* loc, double2* y, bool conj_rows, hipStream_t st);
// translation launch shape: threads per block (64, 128, 256), plus one of
// these flags: the XCD slab order of the blocks (each XCD serves an eighth of
// the targets in tree order), or the node-range order (each XCD serves an
// eighth of the nodes of every target, so the signatures it reads, one eighth
// of each source's, stay in its L2)
constexpr int kTranslateSlab = 0x1000;
constexpr int kTranslateNodes = 0x2000;
constexpr int kTranslateFlags = kTranslateSlab | kTranslateNodes;
// code[q] = 2 slot + flip for interaction entry q = (m, n): D_mn is slot
// `slot` of D at node nu (flip 0) or at the antipodal node (flip 1).
// adjoint: loc_n = sum_m conj(D_mn) sig_m over the entries (n, m) of n.
template <typename T, typename V>
void launch_fmm_translate(int64_t nc, const int64_t* il_off, const int64_t* il, const int64_t* code, bool adjoint,
                          int L, int nu, const V* D, const V* sig, V* loc, int tpb, hipStream_t st);
// Sig_p = sum_children shift * Sig_c (grids coincide)
template <typename T, typename V>
void launch_fmm_up_equal(int64_t np, const int64_t* cbeg, const int64_t* cend, int nu, const V* shift,
                         const V* sigc, V* sigp, hipStream_t st);
// Loc_c += conj(shift) * Loc_p (grids coincide)
template <typename T, typename V>
void launch_fmm_down_equal(int64_t nchild, const int64_t* parent, int nu, const V* shift, const V* locp,
                           V* locc, hipStream_t st);
// F[c][t][mi] = sum_j in[c][t][j] Et[j][mi] (Et: DFT table stored j-major);
// mode 0: input in[c] directly (nt x nj, nj <= 256); mode 1: input conj(shift[c]) * par[parent[c]]
template <typename T, typename V>
void launch_fmm_dft(int64_t nc, int nt, int nj, int nm, const V* in, const V* shift, const int64_t* parent,
                    int mode, const V* E, V* out, hipStream_t st);
// out[c][to][mi] = sum_ti M[to][ti][|m|] in[c][ti][mi], m = mi - mhalf (M stored to-major)
template <typename T, typename V>
void launch_fmm_theta(int64_t nc, int nto, int nti, int nm, int mhalf, const T* M, const V* in, V* out,
                      hipStream_t st);
// up: sigp[p][t][j] = sum_{c in children(p)} shift[c][t,j] sum_mi G[c][t][mi] E[mi][j]
// (nj <= 256, nm <= 256)
template <typename T, typename V>
void launch_fmm_up_idft(int64_t np, const int64_t* cbeg, const int64_t* cend, int nt, int nj, int nm,
                        const V* G, const V* E, const V* shift, V* sigp, hipStream_t st);
// down: locc[c][t][j] += sum_mi K[c][t][mi] E[mi][j]
template <typename T, typename V>
void launch_fmm_down_idft(int64_t nc, int nt, int nj, int nm, const V* K, const V* E, V* locc,
                          hipStream_t st);

// ------------------------------------------------- evaluation grid (FP64) ---
// Per far pair q = (point cluster P, leaf cluster C): X = zp[P] - zc[C],
// coef[q][l] = i^l (2l+1) h_l(k|X|) (l = 0..L) and the unit vector dir[q] = X/|X|.
void launch_grid_coef(int64_t npairs, const int64_t* pair_p, const int64_t* pair_c, const double* zp,
                      const double* zc, double k, int L, double2* coef, double* dir, hipStream_t st);
// loc[P][nu] = sum_{q in far(P)} D_q(nu) (sigA + sigB)[C(q)][nu] with
// D_q(nu) = sum_l coef[q][l] P_l(s_nu . dir[q]) evaluated on the fly.
void launch_grid_translate(int64_t npc, const int64_t* far_off, const int64_t* pair_c, const double2* coef,
                           const double* dir, int L, int nu, const double* s, const double2* sigA,
                           const double2* sigB, double2* loc, hipStream_t st);

}  // namespace bem
