// The opaque bem_mesh object and internal entry points shared by api.cpp,
// solver.cpp and the FMM files.
#pragma once

#include <memory>

#include "common.h"
#include "device.h"

namespace bem {
struct FmmState;                                     // fmm_setup.cpp
void fmm_destroy(FmmState* f);
}  // namespace bem

struct bem_mesh;
namespace bem {
// the quadrilateral records of a mesh as the kernels take them
QuadRecs quad_recs(const bem_mesh* m);
}  // namespace bem

struct bem_mesh {
  bem_options opt{};
  int64_t N = 0;
  bool fmm = false;
  bem::Tree tree;
  bem::Geometry g;                 // tree order
  std::shared_ptr<bem::NearPlan> plan;  // items by target (shared with the host tree it came from)
  bool have_plan_t = false;
  bem::NearPlan plan_t;            // items by source (conjugate transpose)
  int64_t bad_element = -1;

  bem::DevBuf<double> d_geom;
  bem::DevBuf<float> d_geom32;
  // plane quadrilaterals: element -> quadrilateral index, half -> element,
  // halves' geometry (FP64, FP32); empty on triangle meshes
  bem::DevBuf<int64_t> d_qidx, d_hown;
  bem::DevBuf<double> d_hq;
  bem::DevBuf<float> d_hq32;
  bem::DevBuf<int64_t> d_perm;
  bem::DevBuf<int64_t> d_off, d_off_t, d_seg, d_seg_t;
  bem::DevBuf<int32_t> d_order;    // targets by decreasing near-field work
  bem::DevBuf<double> d_rec;       // element records of the quadrature kernels (per wavenumber)
  bem::DevBuf<float> d_rec32;
  double kap = 0.0, kap32 = 0.0;   // their scales
  int n_cu = 256;                  // compute units of the mesh's device
  bem::DevBuf<uint64_t> d_items, d_items_t;
  bem::DevBuf<double> d_duffy_u, d_duffy_w, d_edge_t, d_edge_w;

  // per-problem state
  bool have_problem = false;
  double k = 0.0;
  double gre = 0.0, gim = 0.0;     // coupling gamma
  bool have_beta = false;
  bem::DevBuf<double2> d_beta;     // caller order
  bem::DevBuf<double2> d_cfac;     // tree order, c_j = -i k beta_j
  bem::DevBuf<double2> d_diag;     // tree order, A_ii
  bem::DevBuf<double2> d_vdiag;    // tree order, diagonal of dA/dc

  // launch shapes chosen by bem_autotune, [0] FP64, [1] complex FP32
  int tune_wpb[2] = {4, 4};     // near-field targets per workgroup
  int tune_tpb[2] = {64, 64};   // translation threads per workgroup
  int tune_nwaves[2] = {0, 0};  // resident near-field wavefronts per CU beside the far field (0: one per target)
  int tune_split[2] = {100, 100};  // percent of the near-field targets in the resident launch beside the far
                                   // field; the rest run one wavefront each after the far field, on its stream
  int tune_fork_late[2] = {0, 0};  // leaf translation forked after the leaf level's upward transfer (1) or before (0)

  // captured operator applications of the Krylov driver, [op][precision]
  struct GraphSlot {
    hipGraphExec_t exec = nullptr;
    uint64_t stamp = 0;
    const void* in = nullptr;
    void* out = nullptr;
  };
  GraphSlot graphs[2][2];
  uint64_t problem_stamp = 0;   // bumped by every bem_set_problem
  hipStream_t cap_stream = nullptr;
  // the mesh's stream inside bem_solve_batch (forked from and joined to the
  // caller's stream)
  hipStream_t batch_stream = nullptr;
  hipEvent_t ev_batch = nullptr;

  // the far field runs on a second stream, concurrently with the near field
  // (into d_far), and is added after both finish
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bem::DevBuf<double2> d_far;
  // inside the FMM, the leaf-level translation runs on a third stream beside
  // the upward pass, the upper levels' translations and the downward pass
  hipStream_t leaf_stream = nullptr;
  hipEvent_t ev_leaf_fork = nullptr, ev_leaf_join = nullptr;
  bool capturing = false;  // set while an application is captured into a graph
  // prescribed-pressure (PRES) elements: their unknown is v = dp/dn, so the
  // system's columns there are those of V = dA/dc instead of A
  bem::DevBuf<double> d_pres;       // tree order: 1 on PRES elements, 0 elsewhere
  bem::DevBuf<double2> d_px, d_py;  // masked input and second application
  bool has_pres = false;

  // direct far field (far_direct option): for every operator (far_direct),
  // or for the FP64 operator only, the complex-FP32 one keeping the FMM
  // (far_direct64)
  bool far_direct = false;
  bool far_direct64 = false;
  bem::DevBuf<int32_t> d_elem_leaf;
  bem::DevBuf<int64_t> d_far_off, d_far_beg, d_far_end;
  // groups of up to kFarRows collocation points of one leaf for the forward
  // direct far field (first * 8 + count - 1); far_rows as in bem_options
  bem::DevBuf<int64_t> d_far_grp;
  int far_rows = 0;
  double far_rt2_min[8] = {0};    // r~^2 thresholds of the orders (quad_eps)
  double far_rt2_min32[8] = {0};  // the same for the complex-FP32 operator (quad_eps_mixed)

  // block-Jacobi preconditioner (tree order)
  int64_t nblk = 0;
  int64_t blk_entries = 0;
  bool precond_ready = false;
  int64_t singular_blocks = 0;
  bem::DevBuf<int32_t> d_elem_blk, d_blk_n, d_blk_sing;
  bem::DevBuf<int64_t> d_blk_beg, d_blk_off;
  bem::DevBuf<uint64_t> d_blk_items;  // per row, the near items whose source is in the row's block
  bem::DevBuf<int64_t> d_blk_seg;     // their rule segments (N x 9, as the plan's)
  bem::DevBuf<double2> d_blk_a, d_blk_inv;

  // work vectors (tree order)
  bem::DevBuf<double2> d_x, d_y, d_r, d_b, d_sol, d_tmp;
  bem::DevBuf<double2> d_V, d_w, d_z, d_partial, d_h;

  bem::FmmState* fmm_state = nullptr;
  int fmm_L[16] = {0};     // FP64 operator
  int fmm_L32[16] = {0};   // complex-FP32 operator of the mixed path

  ~bem_mesh() {
    for (auto& row : graphs)
      for (auto& gs : row)
        if (gs.exec) (void)hipGraphExecDestroy(gs.exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (batch_stream) (void)hipStreamDestroy(batch_stream);
    if (ev_batch) (void)hipEventDestroy(ev_batch);
    if (side_stream) (void)hipStreamDestroy(side_stream);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (leaf_stream) (void)hipStreamDestroy(leaf_stream);
    if (ev_leaf_fork) (void)hipEventDestroy(ev_leaf_fork);
    if (ev_leaf_join) (void)hipEventDestroy(ev_leaf_join);
    bem::fmm_destroy(fmm_state);
  }
};

namespace bem {

// tree-order operator application (x_t, y_t device, length N)
void apply_tree(bem_mesh* m, bem_op op, bem_precision prec, const double2* x, double2* y, hipStream_t s);
// part 0: whole operator; 1: diagonal + near field; 2: far field only
// vmode: dA/dc (the matrix that multiplies diag(c)) instead of A
void apply_tree_part(bem_mesh* m, bem_op op, bem_precision prec, int part, const double2* x, double2* y,
                     hipStream_t s, bool vmode = false);

// y = M x with the block-Jacobi preconditioner (M^H for op AH); a copy when
// there is none.  x and y must not alias.
void precondition(bem_mesh* m, bem_op op, const double2* x, double2* y, hipStream_t s);

// far field (FMM or direct quadrature): y += far(x), tree order; no-op
// without a cluster tree
void far_apply(bem_mesh* m, bem_op op, bem_precision prec, const double2* x, double2* y, hipStream_t s,
               bool vmode = false);

// FMM far field: y += far(x), tree order.  No-op if the mesh has no FMM.
void fmm_setup_problem(bem_mesh* m, hipStream_t s);
// vmode: apply dA/dc (the matrix multiplying diag(c)) instead of A
void fmm_apply(bem_mesh* m, bem_op op, bem_precision prec, const double2* x, double2* y, hipStream_t s,
               bool vmode = false);
size_t fmm_bytes(const bem_mesh* m);

// Expansion lengths a tree would get at wavenumber k (FP64 and complex-FP32
// sets), whether the stability cap lowered any of them below the accuracy
// length, and an estimate of the far-field device bytes (translation values,
// signatures, locals, leaf rows; both sets).
struct FmmPlanInfo {
  int levels = 0;
  int L[16] = {0};
  int L32[16] = {0};
  bool capped = false;            // either set
  bool capped64 = false, capped32 = false;
  double bytes = 0.0;
};
FmmPlanInfo fmm_plan_info(const Tree& T, int64_t N, double k, const bem_options& o);

struct SolveResult {
  int iterations = 0;
  int refinements = 0;
  double rel_residual = 0.0;
  bool converged = false;
};
// solve op(A) x = b (op = A or A^H)
SolveResult solve_tree(bem_mesh* m, const double2* b, double2* x, hipStream_t s, bem_op op = BEM_OP_A);
// several independent systems (distinct meshes, each on its own stream),
// their GMRES iterations advanced in lock-step
struct BatchItem {
  bem_mesh* m;
  const double2* b;
  double2* x;
  hipStream_t s;
};
std::vector<SolveResult> solve_tree_batch(const std::vector<BatchItem>& items, bem_op op = BEM_OP_A);

void ensure_transposed_plan(bem_mesh* m, hipStream_t s);

// The FP64 far-field set's leaf level as the evaluation grid reads it (after
// bem_set_problem on a mesh with the FMM): expansion length and grid, plain
// aggregation rows T[j][nu] (tree order), leaf clusters' element ranges.
struct FmmLeafView {
  int L = 0, nu = 0;
  const double* s = nullptr;    // sphere nodes, 3 per node
  const double* w = nullptr;    // weights
  const double2* T = nullptr;   // N x nu
  const int64_t* ebeg = nullptr;
  const int64_t* eend = nullptr;
  int64_t nc = 0;
};
FmmLeafView fmm_leaf_view(bem_mesh* m);
// FP64 leaf aggregation into sig (nc x nu): factor = true multiplies the rows
// by ik s.n_j (cfac not used), false uses the plain rows
void fmm_leaf_aggregate(bem_mesh* m, const double2* x, bool factor, double2* sig, hipStream_t s);
// truncation-stability test of one pair distance X at the FP64 set's leaf
// length: rounding times (2L+1)|h_L(kX)| within l_eps / 10
bool fmm_leaf_pair_stable(const bem_mesh* m, int L, double X);

// field-point kernels' arguments for the mesh's current problem (part 0:
// K = I^H - c I^G, part 1: K = I^G), and the check of their error flag (the
// tree position of an element whose subdivision overflowed, or -1), which
// waits for the stream and throws BEM_E_MESH naming the element
FieldArgs field_args(bem_mesh* m, int64_t npts, int part);
void check_field_error(bem_mesh* m, const int64_t* err, hipStream_t s);

}  // namespace bem
