// Device-side declarations shared by the HIP translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace bem {

constexpr int kMaxRuleOrder = 8;                       // conical rule orders 1..8
constexpr int kRulePoints = 204;                       // sum of m*m for m = 1..8

// Launch helpers (host-callable, defined in the .hip files).
void upload_rule_tables(const double* a, const double* b, const double* w, const int* off);

// Plane quadrilaterals: element j with qidx[j] = q >= 0 is integrated as the
// records N + 2q and N + 2q + 1 (triangles (P0, P1, P2) and (P0, P2, P3));
// hown[r] is the element of record N + r; hq / hq32 hold the halves'
// geometry with the GeomField layout and stride nh = 2 nq.  nh = 0: the mesh
// has triangles only and the arrays are not read.
struct QuadRecs {
  int64_t nh = 0;
  const int64_t* qidx = nullptr;
  const int64_t* hown = nullptr;
  const double* hq = nullptr;
  const float* hq32 = nullptr;
};

struct NearLaunch {
  int64_t N;
  QuadRecs Q;             // integration records of quadrilaterals (items name records)
  const double* geom;     // G_NFIELDS * N, tree order
  const float* geom32;    // same fields in float (mixed path)
  const int64_t* off;     // N + 1
  const int64_t* seg;     // N * 9: start of the order-1..8 items of each target, then its end
  const uint64_t* items;
  const double2* cfac;    // c_j, tree order (nullptr: sound-hard everywhere)
  const double2* diag;    // A_ii, tree order
  const double2* vdiag;   // diagonal of dA/dc: G_ii - gamma/2 (tree order)
  double k;
  double gre, gim;        // coupling gamma
  int wpb;                // targets (wavefronts) per workgroup of the forward kernel: 1, 2, 4 or 8
  const int32_t* order;   // forward kernel: visiting order of the targets (NULL: tree order)
  const double* rec;      // element records for the FP64 kernels (launch_records), scale kap
  const float* rec32;     // element records for the FP32 kernels, scale kap32
  double kap, kap32;      // k (phase in radians) and k / (2 pi) rounded to float (phase in revolutions)
  int64_t nwaves;         // forward kernel: wavefronts launched (0: one per target)
  int64_t first, count;   // forward kernel: the targets at positions first .. first + count - 1 of
                          // the visiting order (count 0: all N)
};

// y = diag x + sum over near items (tree-order vectors), in FP64 or complex
// FP32.  adjoint: conjugate transpose over the transposed item lists (items
// indexed by source), y = conj(diag) x + sum_i conj(K_ij) x_i.  vmode: the
// operator dA/dc instead of A.
void launch_near(const NearLaunch& L, bool fp64, bool adjoint, bool vmode, const double2* x, double2* y,
                 hipStream_t s);

// Far field by direct on-the-fly quadrature: every pair whose leaf clusters
// are admissible (complement of the near list), with the same rule selection
// as the near plan evaluated per pair (order from r~, subdivision while
// r~ < ratio).  far_off/far_beg/far_end: per leaf cluster the element
// intervals (tree order) outside its near clusters.
struct FarLaunch {
  int64_t N;
  QuadRecs Q;
  const double* geom;
  const float* geom32;
  const double2* cfac;
  const int32_t* elem_leaf;
  const int64_t* far_off;
  const int64_t* far_beg;
  const int64_t* far_end;
  double rt2_min[kMaxRuleOrder];  // order m suffices iff r~^2 > rt2_min[m-1] (FP64 kernels)
  double rt2_min32[kMaxRuleOrder];  // the same for the complex-FP32 kernels
  double ratio2;
  int m_max, split_on_cap, max_subdiv;
  double k, gre, gim;
  const double* rec;      // as in NearLaunch
  const float* rec32;
  double kap, kap32;
  // forward operator on triangle meshes: groups of up to kFarRows
  // consecutive collocation points of one leaf, one wavefront each, coded
  // first * 8 + (count - 1); nullptr: one point per wavefront
  const int64_t* grp;
  int64_t ngrp;
};
constexpr int kFarRows = 4;
// y += far(x) (adjoint: y += far^H x; vmode: the dA/dc part), tree order
void launch_far_direct(const FarLaunch& F, bool fp64, bool adjoint, bool vmode, const double2* x, double2* y,
                       hipStream_t s);

struct SelfLaunch {
  int64_t N;
  QuadRecs Q;
  const double* geom;
  const double2* cfac;
  double2* vdiag;         // optional output: G_ii - gamma/2
  const double* duffy_u; const double* duffy_w; int self_n;
  const double* edge_t; const double* edge_w; int edge_pts;
  double k, gre, gim;
};
void launch_self_terms(const SelfLaunch& L, double2* diag, hipStream_t s);

// Per-element records of the quadrature kernels, 16 values per element
// (tree order): v0, e1 = v1 - v0, e2 = v2 - v0 multiplied by the scale, the
// normal, the scaled |e1|^2, |e2|^2, 2 e1.e2 and 2 area.  rec: scale kap
// (FP64), rec32: scale kap32 (FP32).
void launch_records(int64_t N, const double* geom, double kap, double kap32, double* rec, float* rec32,
                    hipStream_t s);
// the same for the n records whose geometry is geom (stride n), written at
// rec + 16 first, rec32 + 16 first (the quadrilaterals' halves)
void launch_records_at(int64_t n, const double* geom, int64_t first, double kap, double kap32, double* rec,
                       float* rec32, hipStream_t s);

// Block-Jacobi preconditioner: the elements (tree order) are partitioned into
// contiguous blocks of at most kMaxBlock elements; block b covers
// [beg[b], beg[b] + n[b]) and its dense n x n matrix (column-major) starts at
// off[b] in the block storage.
constexpr int kMaxBlock = 64;
struct BlockArgs {
  int64_t nblk;
  const int32_t* elem_blk;  // N: block of each element
  const int64_t* beg;       // nblk
  const int32_t* n;         // nblk
  const int64_t* off;       // nblk
  const uint64_t* items;    // per row, the near items with their source in the row's block
  const int64_t* seg;       // N * 9 rule segments of those items (as NearLaunch::seg)
};
// a[off + jl * n + il] = A_(beg + il, beg + jl): diagonal plus the near-field
// entries inside the block, in FP64
void launch_block_assemble(const NearLaunch& L, const BlockArgs& B, double2* a, hipStream_t s);
// inverse of every block by Gauss-Jordan elimination with partial pivoting;
// a block with a zero pivot gets the inverse of its diagonal and sets
// singular[b] = 1
void launch_block_invert(const BlockArgs& B, const double2* a, double2* inv, int32_t* singular, hipStream_t s);
// y = M x with M = blockdiag(inv) (conj_t: M^H); x and y must not alias
void launch_block_apply(int64_t N, const BlockArgs& B, const double2* inv, bool conj_t, const double2* x,
                        double2* y, hipStream_t s);

struct FieldArgs {
  int64_t N;             // elements
  QuadRecs Q;
  int64_t npts;          // field points
  const double* geom;    // tree order
  const double2* cfac;   // c_j (tree order) or NULL
  double k;
  double eps, ratio;     // quadrature tolerance, subdivision ratio
  int m_max, split_on_cap, max_subdiv;
  int part;              // 0: K = I^H - c I^G; 1: K = I^G
  const double2* dpdn;   // k_field only: if set, the scattered field is
                         // tau sum_j I^H_j p_j - I^G_j dpdn_j (tree order) and
                         // cfac and part are not used
  double tau;            // with dpdn: 1 exterior, -1 inside an interior problem
};
// out[f] = pinc[f] + sum_j K_fj p[j] (p in tree order); err[0] receives the
// tree position of an element whose subdivision overflowed
void launch_field(const FieldArgs& A, const double* pts, const double2* p, const double2* pinc, double2* out,
                  int64_t* err, hipStream_t s);
void launch_energy(int64_t n, const double2* p, double* energy, hipStream_t s);
// evaluation grid: near part by element integrals, far part from the point
// clusters' local expansions (points and output in cluster order; A.tau
// gives the sign of the scattered field)
void launch_grid_eval(const FieldArgs& A, const double* pts, const int64_t* pc, const double* zp, int nu,
                      const double* sn, const double* wn, const double2* loc, const int64_t* near_off,
                      const int64_t* near_beg, const int64_t* near_end, const double2* p, const double2* v,
                      const double2* pinc, double2* out, int64_t* err, hipStream_t s);
// v = c p elementwise (c NULL: v = 0)
void launch_cmul(int64_t N, const double2* c, const double2* p, double2* v, hipStream_t s);
// y[j] = sum_f conj(K_fj) g[f] (y in tree order)
void launch_field_adj(const FieldArgs& A, const double* pts, const double2* g, double2* y, int64_t* err,
                      hipStream_t s);
void launch_grad_admittance(int64_t N, double k, double rho_c, const double2* p, const double2* w,
                            const double2* hg, double* grad, hipStream_t s);

void launch_rhs_plane(int64_t N, const double* geom, double k, double gre, double gim,
                      const double* d, double p0re, double p0im, double2* out, hipStream_t s);
void launch_rhs_point(int64_t N, const double* geom, double k, double gre, double gim,
                      const double* x0, double p0re, double p0im, double2* out, hipStream_t s);
void launch_incident(int64_t n, const double* pts, int kind, double k, const double* src, double p0re,
                     double p0im, double2* out, hipStream_t s);
void launch_gather(int64_t N, const int64_t* perm, const double2* src, double2* dst, hipStream_t s);
void launch_scatter(int64_t N, const int64_t* perm, const double2* src, double2* dst, hipStream_t s);
void launch_cfac(int64_t N, const int64_t* perm, const double2* beta_caller, double k, double2* cfac,
                 hipStream_t s);
// v[perm[t]] = -i p[perm[t]] / (k rho_c) where pres[t] != 0 (caller-order p, v;
// tree-order mask): the velocity of PRES elements, whose solution is dp/dn
void launch_velocity_pres(int64_t N, const int64_t* perm, const double* pres, double k, double rho_c,
                          const double2* p, double2* v, hipStream_t s);
void launch_velocity(int64_t N, const double2* beta_caller, double rho_c, const double2* p,
                     double2* v, hipStream_t s);

// Krylov helpers (FP64)
void launch_multidot(int64_t N, int nv, const double2* V, int64_t ldv, const double2* w,
                     double2* partial, int nblk, hipStream_t s);
void launch_reduce_partials(int nv, int nblk, const double2* partial, double2* h, hipStream_t s);
void launch_multiaxpy(int64_t N, int nv, const double2* V, int64_t ldv, const double2* h,
                      double sign, double2* w, hipStream_t s);
void launch_scale_copy(int64_t N, const double2* w, double2 alpha, double2* out, hipStream_t s);
// out[0 .. n) = value (a kernel: no memset node in captured graphs)
void launch_fill_i64(int64_t n, int64_t value, int64_t* out, hipStream_t s);
// out = 0 (a kernel, so that it can sit in a captured graph)
void launch_zero(int64_t N, double2* out, hipStream_t s);
void launch_axpby(int64_t N, double2 a, const double2* x, double2 b, const double2* y, double2* out,
                  hipStream_t s);
// interior problem: turn an exterior application y (of x) into the interior
// one, y = -y + 2 D x (mode: 0 A, 1 A^H, 2 V, 3 V^H, 4 integral part only)
void launch_interior(int64_t N, int mode, double gre, double gim, const double2* cfac, const double2* x,
                     double2* y, hipStream_t s);
// out = x where mask m == keep, else 0; blend: y = z where m == 1 (PRES elements)
void launch_mask(int64_t N, const double* m, int keep, const double2* x, double2* out, hipStream_t s);
void launch_blend(int64_t N, const double* m, double2* y, const double2* z, hipStream_t s);
int multidot_blocks(int64_t N);

}  // namespace bem
