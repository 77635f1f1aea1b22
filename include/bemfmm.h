/*
 * bemfmm.h -- C ABI of the MI355X (gfx950) Burton-Miller BEM / multilevel FMM
 * library.
 *
 * The library solves the exterior Helmholtz problem on a closed surface made
 * of flat triangles with constant elements and collocation at the centroids
 * (arXiv 2312.00005, Sec. 2.2-2.3), in the Burton-Miller form of Eq. (SystemI)
 * with tau = 1 and coupling gamma = i/k (Sec. 2.5):
 *
 *   (phi - gamma v)/2 - (H - gamma E) phi + (G - gamma H') v = phi_inc - gamma v_inc
 *
 * Per element j the boundary condition is v_j = c_j phi_j with c_j = 0 on a
 * sound-hard element (the default of the paper's mesh appendix) and
 * c_j = -tau i k beta_j for an admittance element, beta = rho c Y: the
 * normal velocity along the outward mesh normal is v = -tau Y p (absorbing on
 * an exterior surface, tau = 1; on an interior problem, tau = -1, the
 * condition of the duct of Sec. 5.3).  The unknown may be read as surface
 * pressure p; all source amplitudes are pressure amplitudes.
 *
 * The operator A is applied as the near field (direct singular,
 * hypersingular, quasi-singular and regular quadrature, Sec. 3.1, evaluated
 * on the fly on every application) plus the far field of a multilevel fast
 * multipole method on the paper's cluster tree (Sec. 3.3): aggregation of
 * leaf elements to signatures on unit-sphere quadrature points, band-limited
 * interpolation between levels, diagonal translation by the truncated
 * expansion of Eq. (FMMBase), anterpolation and disaggregation.
 *
 * Conventions (all functions):
 *   - SI units; k is the wavenumber in rad/m.
 *   - bem_c128 is layout-compatible with C99 double complex,
 *     std::complex<double> and a torch.complex128 element.
 *   - Vectors indexed by element follow the caller's triangle order.
 *   - "device" pointers are HIP device pointers on the current device
 *     (e.g. tensor.data_ptr() of a CUDA/HIP tensor); "host" pointers are
 *     ordinary CPU memory.  Buffers are owned by the caller; the library owns
 *     only the memory held by a bem_mesh and releases it in bem_mesh_destroy.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     work on it and return; bem_mesh_create and bem_solve return only when
 *     their result is complete.
 *   - Every function returns a bem_status; on failure bem_last_error() gives a
 *     thread-local message valid until the next call on the same thread.
 *     Nothing is thrown across this boundary.
 *   - A bem_mesh is not thread-safe.  Calls from several host threads at
 *     once, even on different meshes, are not supported: a run with two
 *     threads solving on two meshes ended in a host crash whose cause is not
 *     known.  Use the library from one host thread per device at a time.
 */
#ifndef BEMFMM_H
#define BEMFMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } bem_c128;

typedef enum {
  BEM_OK = 0,
  BEM_E_ARG = 1,     /* invalid argument (NULL pointer, size, NaN, unknown preset) */
  BEM_E_MESH = 2,    /* degenerate triangle, or more nested subdivisions than
                        allowed (Sec. 4.1 "subdivision loop" error); see
                        bem_mesh_bad_element() */
  BEM_E_NOCONV = 3,  /* iterative solver did not reach the tolerance; the
                        outputs hold the last iterate */
  BEM_E_HIP = 4,     /* a HIP runtime call failed */
  BEM_E_OOM = 5,     /* device or host allocation failed */
  BEM_E_STATE = 6    /* call out of order (e.g. apply before set_problem) */
} bem_status;

typedef enum { BEM_PREC_FP64 = 0, BEM_PREC_MIXED = 1 } bem_precision;

/* Operator selector of bem_apply. */
typedef enum {
  BEM_OP_A = 0,   /* y = A x                          */
  BEM_OP_AH = 1   /* y = A^H x (conjugate transpose)  */
} bem_op;

/* Warning bits of bem_solve_info.warnings (computation continues). */
#define BEM_WARN_COARSE_MESH 1u  /* fewer than 6 elements per wavelength (Sec. 2.2) */
#define BEM_WARN_LARGE_L 2u      /* an expansion length above 30 (Sec. 4.2)      */
#define BEM_WARN_NOT_CONVERGED 4u/* iterative solver stopped at its cap (Sec. 3.2) */

typedef struct bem_options {
  int32_t use_fmm;          /* 0: every pair by direct quadrature (dense
                               operator applied on the fly); 1: FMM          */
  int32_t levels;           /* number of tree levels (root = 1) when use_fmm */
  int32_t leaf_size;        /* target elements per leaf cluster              */
  double root_box_edge;     /* root sub-box edge; 0 = derived from levels and
                               leaf_size (Sec. 3.3.4)                        */
  double admissibility;     /* far if |z_i - z_j| > admissibility (r_i + r_j);
                               2/sqrt(3) in Eq. (Farfieldcond)               */
  int32_t l_mode;           /* 0: L from Eq. (FMMTruncation) alone;
                               1: also an accuracy term (see l_eps)          */
  double l_factor;          /* 1.8 in Eq. (FMMTruncation)                    */
  int32_t l_min;            /* lower bound of L (8 in Eq. (FMMTruncation))   */
  double l_eps;             /* target accuracy of the expansion (l_mode 1)   */
  int32_t t_order;          /* order of the triangle rule for aggregation    */
  double quad_eps;          /* a-priori quadrature tolerance (1e-3, Sec. 3.1.4) */
  int32_t quad_m_max;       /* maximum Gauss order (6, Sec. 3.1.4)           */
  int32_t quad_split_on_cap;/* 1: split instead of capping the order (Sec. 5.1.2) */
  double subdiv_ratio;      /* split while r~ < subdiv_ratio (1.3, Sec. 3.1.3) */
  int32_t max_subdiv;       /* nested split limit (15, Sec. 4.1)             */
  int32_t self_n;           /* Duffy rule order per direction (4, Sec. 3.1.1) */
  int32_t edge_parts;       /* parts per edge for E_ii (4, Sec. 3.1.2)        */
  int32_t edge_gauss;       /* Gauss points per part (3, Sec. 3.1.2)          */
  bem_precision precision;  /* arithmetic of the inner operator in bem_solve */
  int32_t gmres_restart;    /* Krylov dimension before restart                */
  int32_t gmres_maxit;      /* iteration cap (250 as in Sec. 3.2)             */
  double gmres_tol;         /* relative residual target                       */
  int32_t refine_maxit;     /* outer refinement steps (mixed precision)      */
  double inner_tol;         /* inner GMRES tolerance (mixed precision),
                               relative to the current FP64 residual; an inner
                               solve never goes below half of gmres_tol |b| */
  double l_eps_mixed;       /* expansion accuracy of the complex-FP32 operator;
                               its L is also capped so that FP32 rounding times
                               (2L+1)|h_L(k X_min)| stays below l_eps_mixed/10 */
  int32_t precond;          /* right preconditioner of GMRES (the role of
                               the near-field preconditioning of Sec. 3.2):
                               0 none; 1 block Jacobi -- the dense near-field
                               blocks of the leaf clusters (split into pieces
                               of at most 64 elements) inverted per
                               frequency; 2 diagonal (Jacobi) scaling */
  double gamma_re;          /* Burton-Miller coupling                        */
  double gamma_im_k;        /*   gamma = gamma_re + i gamma_im_k / k; the
                               paper's gamma = i/k is (0, 1) (Sec. 2.5).
                               Any gamma with a non-zero imaginary part gives
                               a uniquely solvable system; on non-spherical
                               bodies at ka >> 1, (0, -1) places the spectrum
                               of the discrete operator in the right
                               half-plane and Krylov iterations converge far
                               faster.  gamma_im_k = 0 is BEM_E_ARG. */
  int32_t far_direct;       /* 1: keep the cluster tree and near plan but
                               evaluate the far field by direct quadrature of
                               every admissible pair (same rules as the near
                               plan, chosen per pair on the fly; nothing
                               stored) instead of the FMM -- for frequencies
                               where the expansion is unstable (k X_min small,
                               Sec. 3.3.1) or too long.  2: the FP64 operator
                               integrates the far field directly and the
                               complex-FP32 operator keeps the FMM -- for the
                               mixed path at frequencies where only the FP64
                               expansion lengths are capped (the FP64
                               refinement residuals then hold the solution's
                               accuracy, the FP32 inner solves only need a good
                               operator).  Needs use_fmm = 1. */
  int32_t use_graphs;       /* 1: bem_solve / bem_solve_adjoint replay the
                               operator application (near field and far field
                               kernels) of each GMRES iteration as a captured
                               HIP graph; recaptured after bem_set_problem */
  int32_t level_rows;       /* far-field level transfer: 0 = band-limited
                               interpolation / anterpolation between levels
                               (leaf rows only); 1 = the paper's explicit
                               element-to-cluster rows T(l), S(l) stored on
                               every level with interaction pairs (Sec. 3.3.4;
                               memory N * sum_l 2 L_l^2 per row set) */
  int32_t solver;           /* 0: restarted GMRES (CGS2 orthogonalisation);
                               1: conjugate gradient squared, the paper's
                               iterative solver (Sec. 3.2); both right
                               preconditioned, gmres_maxit caps iterations */
  int32_t near_waves_per_cu;/* forward near-field kernel: 0 = one wavefront
                               per collocation point, all launched at once;
                               n in [1, 64] = n resident wavefronts per compute
                               unit, each looping over collocation points, so
                               that the far-field kernels on the side stream
                               find free wavefront slots (a tuning choice;
                               results are identical) */
  double quad_eps_mixed;    /* quadrature tolerance (Sec. 3.1.4 estimates) of
                               the direct far field (far_direct = 1) in the
                               complex-FP32 operator, whose pair orders are
                               chosen on the fly; the FP64 operator and every
                               near-field plan use quad_eps (tight / mixed:
                               equal to quad_eps, so that the two operators
                               differ by rounding only) */
  int32_t interior;         /* 0: exterior problem (tau = 1 in Eq. (SystemI));
                               1: interior problem (tau = -1: every integral
                               term negated, the jump term (phi - gamma v)/2
                               kept; the mesh normals still point out of the
                               object, i.e. out of the fluid; admittance then
                               means v = +Y p, c = +i k beta).  Interior
                               meshes use no block-Jacobi preconditioner and
                               refuse bem_field, bem_field_adjoint and
                               bem_grad_admittance (exterior representation
                               formula); bem_field_pv evaluates points inside
                               the fluid. */
  int32_t translate_shape;  /* far-field translation launch: threads per
                               block 64, 128 or 256 (0: 64), plus 4096 for the
                               XCD slab order of the blocks (each of the 8 XCDs
                               serving an eighth of a level's targets in tree
                               order) or 8192 for the node-range order (each
                               XCD serving an eighth of the sphere nodes of
                               every target); a tuning choice, results are
                               identical; bem_autotune replaces it */
  int32_t near_split;       /* with near_waves_per_cu > 0: percent (1-99) of the
                               collocation points whose near field runs in the
                               resident grid beside the far field; the rest run
                               one wavefront each on the far field's stream
                               after it, at full occupancy (0 or 100: all in
                               the resident grid).  A tuning choice, results
                               are identical; bem_autotune replaces it */
  int32_t far_rows;         /* direct far field (far_direct), forward operator
                               on triangle meshes: collocation points per
                               wavefront, 1 or 4 (0: 4 in the FP64 operator, 1
                               in the complex-FP32 one).  With 4, consecutive
                               points of one leaf cluster share every source
                               element's loads.  A tuning choice: the same
                               sums in the same order, equal to rounding */
} bem_options;

typedef struct bem_solve_info {
  int32_t iterations;       /* total inner Krylov iterations                 */
  int32_t refinements;      /* outer refinement steps (mixed)                */
  int32_t levels;           /* tree levels (0 without FMM)                   */
  int32_t L[16];            /* expansion length per level, root first        */
  int32_t clusters[16];     /* clusters per level, root first                */
  int64_t near_pairs;       /* near element pairs, self pairs included       */
  int64_t near_items;       /* quadrature items (sub-triangles) per apply    */
  int64_t quad_points;      /* near-field quadrature points per apply        */
  double rel_residual;      /* final ||b - A x|| / ||b|| (FP64 operator)      */
  uint32_t warnings;        /* BEM_WARN_* bits                                */
  int32_t L_mixed[16];      /* expansion length per level of the complex-FP32
                               operator (mixed path), root first             */
} bem_solve_info;

typedef struct bem_mesh bem_mesh;

/* Device allocator of the library's own memory (plan, per-frequency state,
 * work vectors).  alloc_fn(bytes, ctx) returns device memory on the current
 * device (NULL on failure: the calling entry point then returns BEM_E_OOM);
 * free_fn(ptr, bytes, ctx) takes back what alloc_fn returned, with the same
 * byte count.  The memory is used on the streams the caller passes and on
 * the library's internal streams; before a block is returned the library
 * waits for the device (hipDeviceSynchronize), so free_fn may hand it out
 * again at once.  A typical pair is PyTorch's caching allocator.
 *
 * bem_set_allocator sets the pair for the whole process (both NULL restores
 * hipMalloc / hipFree; one NULL is BEM_E_ARG).  Every buffer keeps the pair it
 * was allocated with, so the pair may change between meshes; it must stay
 * callable until every buffer allocated through it is released
 * (bem_mesh_destroy).  Not to be called while another thread is inside the
 * library. */
typedef void* (*bem_alloc_fn)(size_t bytes, void* ctx);
typedef void (*bem_free_fn)(void* ptr, size_t bytes, void* ctx);
bem_status bem_set_allocator(bem_alloc_fn alloc_fn, bem_free_fn free_fn, void* ctx);

/* Fill *o with a named preset: "paper" (the paper's defaults), "tight"
 * (higher-accuracy quadrature and expansion, FP64) or "mixed" ("tight" with
 * complex-FP32 inner operator and FP64 refinement).  Unknown name: BEM_E_ARG. */
bem_status bem_options_default(bem_options* o, const char* preset);

/* Build the mesh plan: element geometry, cluster tree (Sec. 3.3.2-3.3.4),
 * interaction lists, near-field pairs and their frequency-independent
 * quadrature plan (Sec. 3.1.3-3.1.4), and upload it to the current device.
 *   xyz : host, double[n_nodes][3]
 *   tri : host, int32[n_tri][3], 0-based node indices, counter-clockwise seen
 *         from outside (the paper's mesh appendix)
 * The uploads run on `stream`.  Blocking: returns when the plan is on the
 * device.  BEM_E_MESH for a zero-area triangle or a subdivision overflow. */
bem_status bem_mesh_create(int64_t n_nodes, const double* xyz, int64_t n_tri,
                           const int32_t* tri, const bem_options* o,
                           void* stream, bem_mesh** out);

/* The same for a mesh of flat triangles and plane quadrilaterals (Sec. 2.2):
 *   el : host, int32[n_el][4], 0-based node indices counter-clockwise seen
 *        from outside; el[e][3] < 0 marks a triangle
 * A quadrilateral's collocation node is the mean of its four vertices (Sec.
 * 2.3) and its normal lies along (P2 - P0) x (P3 - P1); it is integrated as
 * the two triangles (P0, P1, P2) and (P0, P2, P3), each with the rules of a
 * triangle (the paper's m x m product rule gives the same integral to the
 * quadrature tolerance), and its singular integral by eight Duffy
 * sub-triangles around the node (Sec. 3.1.1) and its four edges (Sec.
 * 3.1.2).  Every later call takes vectors of n_el values, one per element.
 * BEM_E_MESH (bem_mesh_bad_element names it) for a quadrilateral whose
 * vertices lie more than 1e-8 of its longer diagonal off their mean plane,
 * one that is not convex, or a degenerate element. */
bem_status bem_mesh_create_elements(int64_t n_nodes, const double* xyz, int64_t n_el,
                                    const int32_t* el, const bem_options* o,
                                    void* stream, bem_mesh** out);

/* Element index (caller order) that caused the last BEM_E_MESH, or -1. */
int64_t bem_mesh_bad_element(const bem_mesh* m);

/* Per-frequency setup: wavenumber k > 0 and per-element normalised
 * admittance beta (device bem_c128[n_tri], or NULL for sound-hard
 * everywhere).  Computes the singular self terms, expansion lengths, sphere
 * grids, interpolation and translation data (Sec. 3.3.1, Sec. 4.2). */
bem_status bem_set_problem(bem_mesh* m, double k, const bem_c128* beta,
                           void* stream);

/* Right-hand side b = p_inc - gamma dp_inc/dn at the centroids (Sec. 2.4):
 * plane wave P0 exp(i k d.x) with unit direction d, or point source
 * P0 exp(i k R)/(4 pi R) at x0.  rhs: device bem_c128[n_tri]. */
bem_status bem_rhs_plane_wave(bem_mesh* m, const double d[3], bem_c128 P0,
                              bem_c128* rhs, void* stream);
bem_status bem_rhs_point_source(bem_mesh* m, const double x0[3], bem_c128 P0,
                                bem_c128* rhs, void* stream);

/* One operator application y = A x or y = A^H x (device vectors of n_tri),
 * in FP64 or in the mixed path's complex-FP32 arithmetic (self terms FP64). */
bem_status bem_apply(bem_mesh* m, bem_op op, bem_precision prec,
                     const bem_c128* x, bem_c128* y, void* stream);

/* The two parts of one application, for measurement and testing:
 * part = 1: y = (diagonal + near field) x only; part = 2: y = far field
 * (FMM) x only (zero without FMM); part = 0 is bem_apply. */
bem_status bem_apply_part(bem_mesh* m, bem_op op, bem_precision prec, int part,
                          const bem_c128* x, bem_c128* y, void* stream);

/* y = V x or y = V^H x with V = dA/dc, the matrix that multiplies diag(c) in
 * A(c) = A(0) + V diag(c) (Eq. (SystemI)): V_ij = G_ij - gamma H'_ij off the
 * diagonal and G_ii - gamma/2 on it.  Used by admittance gradients:
 * dA/dbeta_e = -i k V e_e e_e^T.  Device vectors of n_tri. */
bem_status bem_apply_dc(bem_mesh* m, bem_op op, bem_precision prec,
                        const bem_c128* x, bem_c128* y, void* stream);

/* Prescribed pressure (PRES condition of the input description, appendix;
 * p = 0 makes an element sound soft).  elems: host int64[n] element indices
 * (caller's order), n = 0 clears the set.  On these elements the pressure is
 * known and the unknown of bem_solve becomes v = dp/dn: the system's columns
 * there are those of V = dA/dc (see bem_apply_dc) instead of A, every
 * application of A then runs A and V once each, admittance on these elements
 * is ignored and no block-Jacobi factors are used.  Invalidates the problem:
 * call bem_set_problem afterwards.  Errors: BEM_E_ARG for an index outside
 * the mesh. */
bem_status bem_set_pressure_elements(bem_mesh* m, int64_t n, const int64_t* elems, void* stream);

/* rhs <- rhs - A p_bar over the PRES elements (their known pressures moved to
 * the right-hand side; p_bar: device bem_c128[n_tri] in the caller's order,
 * read only on PRES elements).  FP64 operator.  BEM_E_STATE without PRES
 * elements or before bem_set_problem. */
bem_status bem_rhs_pressure(bem_mesh* m, const bem_c128* pbar, bem_c128* rhs, void* stream);

/* Prescribed normal particle velocities (VELO condition of the input
 * description, appendix; may be combined with ADMI): with v = c phi + v_bar
 * and v_bar = i k rho_c u in Eq. (SystemI), the known part moves to the
 * right-hand side:  rhs <- rhs - i k rho_c V u,  V = dA/dc as in
 * bem_apply_dc, applied with the FP64 operator.  u: device bem_c128[n_tri]
 * (outward normal velocity, 0 where not prescribed), caller's element order;
 * rhs: device bem_c128[n_tri], updated in place.  Uses k of the problem;
 * rho_c > 0 or BEM_E_ARG.  The velocity that bem_solve reports (-Y p) does
 * not include u. */
bem_status bem_rhs_velocity(bem_mesh* m, const bem_c128* u, double rho_c, bem_c128* rhs,
                            void* stream);

/* Solve A^H x = rhs (the adjoint system of an admittance gradient) with the
 * same GMRES / refinement settings as bem_solve.  Blocking; info may be NULL. */
bem_status bem_solve_adjoint(bem_mesh* m, const bem_c128* rhs, bem_c128* x_out,
                             bem_solve_info* info, void* stream);

/* Incident pressure at arbitrary points (Sec. 2.4): kind 0 plane wave
 * P0 exp(i k d.x) with d = src (normalised; zero is BEM_E_ARG), kind 1 point
 * source P0 exp(i k R)/(4 pi R), R = |x - src|.  pts: device double[n_pts][3];
 * out: device bem_c128[n_pts]; src is host memory.  Uses k of the problem. */
bem_status bem_incident_field(bem_mesh* m, int kind, const double src[3],
                              bem_c128 P0, int64_t n_pts, const double* pts,
                              bem_c128* out, void* stream);

/* Exterior pressure at field points from the representation formula
 * (Eq. (BIE_I) with lambda = 1, tau = 1):
 *   p_out[f] = p_inc[f] + sum_j (I^H(x_f, G_j) - c_j I^G(x_f, G_j)) p_surf[j],
 * element integrals by the quasi-singular / regular rules of Sec. 3.1.3-3.1.4
 * chosen per (point, element) pair.
 *   pts    : device double[n_pts][3] (outside the body)
 *   p_surf : device bem_c128[n_tri]; p_inc: device bem_c128[n_pts] or NULL
 *   p_out  : device bem_c128[n_pts]
 *   energy : device double[1] receiving sum_f |p_out[f]|^2, or NULL
 * n_pts = 0 is allowed (pts, p_inc, p_out may then be NULL; energy = 0).
 * BEM_E_MESH if a point is so close to an element that subdivision overflows.
 * The normal derivative is taken as c_j p_j (sound-hard or admittance
 * elements): a mesh with PRES elements is BEM_E_STATE, and a prescribed
 * velocity (bem_rhs_velocity) is not included -- use bem_field_pv for both. */
bem_status bem_field(bem_mesh* m, int64_t n_pts, const double* pts,
                     const bem_c128* p_surf, const bem_c128* p_inc,
                     bem_c128* p_out, double* energy, void* stream);

/* bem_field for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, results and errors as bem_field (p_out identical bit for
 * bit; the energy summed in a different, fixed order), but no hipMalloc,
 * hipFree or other allocation.  Its error flag and the partial sums of the
 * energy live in a fixed device array (8 KiB) that each GPU holds until the
 * process ends; n_pts above 4194304 is BEM_E_ARG.  Every call on one GPU
 * shares that array: calls that overlap in time on one GPU race.  Like
 * bem_field it waits for `stream` before returning (the error check). */
bem_status bem_field_noalloc(bem_mesh* m, int64_t n_pts, const double* pts,
                             const bem_c128* p_surf, const bem_c128* p_inc,
                             bem_c128* p_out, double* energy, void* stream);

/* Exterior pressure from the representation formula with the surface
 * pressure and its normal derivative given separately (Eq. (BIE_I),
 * lambda = 1, tau = 1; any boundary condition):
 *   p_out[f] = p_inc[f] + sum_j (I^H(x_f, G_j) p_surf[j] - I^G(x_f, G_j) dpdn_surf[j])
 *   dpdn_surf : device bem_c128[n_tri], dp/dn on the outward normal: c_j p_j
 *               on admittance / sound-hard elements, plus i k rho_c u_j where a
 *               normal velocity u is prescribed, and the solution of bem_solve
 *               on PRES elements (whose p_surf is the prescribed pressure).
 * On an interior mesh (option interior) the points lie inside the fluid and
 * the sum is negated (tau = -1 in Eq. (BIE_I); the mesh normals point out of
 * the fluid).  Other arguments, rules and errors as bem_field. */
bem_status bem_field_pv(bem_mesh* m, int64_t n_pts, const double* pts,
                        const bem_c128* p_surf, const bem_c128* dpdn_surf,
                        const bem_c128* p_inc, bem_c128* p_out, double* energy,
                        void* stream);

/* Conjugate transpose of the field map: y_surf[j] = sum_f conj(K_fj) g[f] with
 * K = I^H - c I^G (part 0) or K = I^G alone (part 1).  g: device
 * bem_c128[n_pts]; y_surf: device bem_c128[n_tri].  BEM_E_STATE on a mesh
 * with PRES elements (the map assumes dp/dn = c p). */
bem_status bem_field_adjoint(bem_mesh* m, int64_t n_pts, const double* pts,
                             const bem_c128* g, int part, bem_c128* y_surf,
                             void* stream);

/* Gradient of J = sum_f |p_f|^2 with respect to the per-element admittance
 * Y_e (beta = rho_c Y) from one adjoint solve:
 *   grad[e] = 2 Re{ -i k rho_c p_e ( -conj(w_e) - conj(h_e) ) }
 * where p solves A p = b, w = V^H mu (bem_apply_dc, op A^H) with
 * A^H mu = M^H p_field, and h = (I^G)^H p_field (bem_field_adjoint, part 1).
 * All inputs device bem_c128[n_tri]; grad: device double[n_tri].
 * BEM_E_STATE on a mesh with PRES elements. */
bem_status bem_grad_admittance(bem_mesh* m, const bem_c128* p, const bem_c128* w,
                               const bem_c128* hg, double rho_c, double* grad,
                               void* stream);

/* Choose launch shapes by timing them on this mesh and problem: near-field
 * targets per workgroup (1, 2, 4, 8) on the near field alone and, with the
 * cluster tree, the resident near-field wavefronts per compute unit while the
 * far field runs beside it (0, 8, 12, 16, 24; see near_waves_per_cu) jointly
 * with the translation threads per workgroup (64, 128, 256; FMM only) and the
 * point where the leaf-level translation leaves the level chain for a stream
 * of its own (right after aggregation, or after the leaf level's transfer to
 * the level above) on whole applications, then the translation blocks in XCD
 * slab order (each of the 8 XCDs serving an eighth of the targets in tree
 * order, so that the source signatures neighbouring targets share stay in
 * one L2) and in XCD node-range order (each XCD serving an eighth of every
 * target's sphere nodes), each at 64, 128 and 256 threads per workgroup,
 * then the share of near-field targets kept beside the far field (see
 * near_split), for the FP64 and the complex-FP32 operator.  Results are kept
 * in the mesh and used by every later application; near_wpb, translate_tpb
 * (threads per workgroup + 4096 for the slab order, + 8192 for the node-range
 * order) and near_waves (host int32[2]: FP64, FP32) receive them and may be
 * NULL.  Runs about 900 operator applications or parts on the stream;
 * results are unchanged by the choice (each output keeps its owner and
 * summation order). */
bem_status bem_autotune(bem_mesh* m, int32_t* near_wpb, int32_t* translate_tpb,
                        int32_t* near_waves, void* stream);

/* Solve A p = rhs by GMRES (FP64 Krylov vectors and residuals; with
 * precision MIXED an FP64 outer refinement around a complex-FP32 inner
 * operator).  p_out: device bem_c128[n_tri]; v_out (may be NULL): normal
 * velocity v = -beta/(rho_c) p.  On PRES elements (bem_set_pressure_elements)
 * p_out holds the unknown there, dp/dn, and v_out = dp/dn / (i k rho_c).
 * A prescribed velocity u (bem_rhs_velocity) is not added to v_out.
 * info: host, may be NULL.  Blocking.
 * BEM_E_NOCONV if the tolerance was not reached (outputs still written). */
bem_status bem_solve(bem_mesh* m, const bem_c128* rhs, bem_c128* p_out,
                     bem_c128* v_out, double rho_c, bem_solve_info* info,
                     void* stream);

/* Solve n independent systems A_i p_i = rhs_i, one per mesh (typically the
 * frequencies of a sweep, each mesh set up with bem_set_problem at its own
 * wavenumber), with the settings of bem_solve.  The GMRES iterations of all
 * systems advance in lock-step, each system on an internal stream of its
 * mesh forked from `stream` after the caller's prior work: while one
 * system's Gram-Schmidt coefficients travel to the host, the kernels of the
 * others run.  Arrays of n pointers (host arrays of device pointers):
 *   meshes : distinct meshes (a mesh twice is BEM_E_ARG)
 *   rhs, p_out : device bem_c128[n_tri of that mesh]
 *   v_out  : NULL, or an array whose entries are NULL or device
 *            bem_c128[n_tri] (velocity as in bem_solve; rho_c > 0 then)
 *   infos  : host bem_solve_info[n] or NULL
 * Blocking: returns when every system is solved and `stream` has joined the
 * internal streams.  BEM_E_NOCONV if any system stopped before its tolerance
 * (all outputs written); BEM_E_STATE if a mesh has no problem set.  With the
 * CGS solver (solver = 1) the systems are solved one after another. */
bem_status bem_solve_batch(int32_t n, bem_mesh* const* meshes,
                           const bem_c128* const* rhs, bem_c128* const* p_out,
                           bem_c128* const* v_out, double rho_c,
                           bem_solve_info* infos, void* stream);

/* Launch shapes in use (host int32[2] each: FP64, complex FP32; any pointer
 * may be NULL): near-field targets per workgroup, translation shape (as
 * translate_shape), resident near-field wavefronts per compute unit and the
 * near-field split (as near_split).  Host only. */
bem_status bem_mesh_launch_shapes(const bem_mesh* m, int32_t* near_wpb, int32_t* translate_shape,
                                  int32_t* near_waves, int32_t* near_split);

/* Mesh statistics (host outputs; any pointer may be NULL). */
bem_status bem_mesh_stats(const bem_mesh* m, int32_t* levels, int32_t* clusters,
                          int64_t* near_pairs, int64_t* near_items,
                          int64_t* quad_points);

/* Device bytes held by the mesh plan and the current problem. */
size_t bem_workspace_bytes(const bem_mesh* m);

void bem_mesh_destroy(bem_mesh* m);

/* ---- host-only inspection of the frequency-independent plan -------------
 * bem_tree_build runs the same geometry, cluster-tree and near-field-plan
 * construction as bem_mesh_create but touches no device; it exists so that
 * the tree and plan can be inspected and tested without a GPU.  The near
 * plan is built on the first bem_tree_plan_stats call (which then reports
 * its errors, e.g. BEM_E_MESH for too many nested subdivisions); the tree
 * queries and bem_tree_fmm_lengths need only the tree.  Levels are
 * numbered from the root (0).  Arrays are written by the caller-sized output
 * pointers (any may be NULL): z[3 nc], r[nc], ebeg/eend/parent[nc] (element
 * ranges in tree order; parent index on the level above, -1 at the root),
 * il_off/near_off[nc + 1] and il/near (cluster indices, CSR). */
typedef struct bem_tree bem_tree;
bem_status bem_tree_build(int64_t n_nodes, const double* xyz, int64_t n_tri,
                          const int32_t* tri, const bem_options* o, bem_tree** out);
int32_t bem_tree_levels(const bem_tree* t);
bem_status bem_tree_level(const bem_tree* t, int32_t level, int64_t* nc,
                          int64_t* n_il, int64_t* n_near);
bem_status bem_tree_level_data(const bem_tree* t, int32_t level, double* z, double* r,
                               int64_t* ebeg, int64_t* eend, int64_t* parent,
                               int64_t* il_off, int64_t* il, int64_t* near_off,
                               int64_t* near);
/* perm[t] = caller index of the element at tree position t (host int64[n_tri]) */
bem_status bem_tree_perm(const bem_tree* t, int64_t* perm);
/* near pairs (self included), quadrature items and points of one application */
bem_status bem_tree_plan_stats(const bem_tree* t, int64_t* pairs, int64_t* items,
                               int64_t* points);
/* Expansion lengths the tree would get at wavenumber k under options o (the
 * admissibility and length rule of o; Eq. (FMMTruncation) and the stability
 * cap): L[level] for the FP64 operator, L32[level] for the complex-FP32 one
 * (both host int32[levels]), *capped: bit 0 set if the cap lowered any FP64
 * length below the accuracy-driven one, bit 1 the same for the complex-FP32
 * lengths (the expansion is then less accurate than asked: k X_min too
 * small, Sec. 3.3.1), *bytes = estimated far-field device memory
 * of bem_set_problem.  Any output may be NULL.  BEM_E_STATE for a tree built
 * without use_fmm. */
bem_status bem_tree_fmm_lengths(const bem_tree* t, double k, const bem_options* o,
                                int32_t* L, int32_t* L32, int32_t* capped,
                                double* bytes);

void bem_tree_destroy(bem_tree* t);

/* A mesh on a host tree's geometry, cluster tree and near plan (the plan is
 * built here if bem_tree_plan_stats has not built it yet), equal to
 * bem_mesh_create on the tree's mesh and options but without building the
 * plan again: for several meshes of one tree that differ in their far-field
 * method, precision, solver or launch options (a frequency sweep).  The
 * options' tree and plan fields (use_fmm, levels, leaf_size, root_box_edge,
 * admissibility, quad_eps, quad_m_max, quad_split_on_cap, subdiv_ratio,
 * max_subdiv) must equal the tree's, else BEM_E_ARG.  The mesh copies what it
 * needs; the tree may be destroyed afterwards. */
bem_status bem_mesh_create_from_tree(const bem_tree* t, const bem_options* o, void* stream,
                                     bem_mesh** out);

/* ---- evaluation grid: pressure at many field points with the FMM ----------
 * The paper's evaluation points (output appendix; the sphere benchmark of
 * Sec. 5.1 uses 24874 of them): the points are grouped into clusters no
 * larger than the mesh's leaf clusters; pairs of a point cluster and a leaf
 * cluster that pass the admissibility test (and the stability test of the
 * FP64 expansion lengths) are evaluated through the leaf signatures, the
 * translation operator of Eq. (FMMBase) (evaluated on the fly from its
 * Legendre series) and a local expansion about the point cluster; the other
 * pairs by the element integrals of bem_field_pv.  Accuracy: that of the FP64
 * far field (l_eps).  Needs a mesh built with use_fmm = 1 and far_direct = 0.
 *   bem_grid_create: pts host double[n_pts][3] (copied); the grid keeps a
 *     pointer to the mesh, which must outlive it.
 *   bem_grid_eval: p_surf, dpdn_surf (NULL: c p, not allowed with PRES
 *     elements), p_inc (NULL: no incident field) and p_out as in
 *     bem_field_pv (device vectors, caller's element / point order); energy
 *     as in bem_field.  Per wavenumber the split into far and near pairs is
 *     rebuilt on the host at the first evaluation.  Blocking (error check).
 *   bem_grid_stats: point clusters, far pairs, near elements summed over the
 *     point clusters (of the last evaluated problem). */
typedef struct bem_grid bem_grid;
bem_status bem_grid_create(bem_mesh* m, int64_t n_pts, const double* pts, bem_grid** out);
bem_status bem_grid_eval(bem_grid* g, const bem_c128* p_surf, const bem_c128* dpdn_surf, const bem_c128* p_inc,
                         bem_c128* p_out, double* energy, void* stream);
bem_status bem_grid_stats(const bem_grid* g, int64_t* point_clusters, int64_t* far_pairs,
                          int64_t* near_elements);
void bem_grid_destroy(bem_grid* g);

/* ---- the paper's automatic choice of method (Sec. 3.3.4, Fig. FMMChange) --
 * Methods in the numbering of the paper's input description (FMM_type):
 * conventional BEM without FMM, single-level FMM, multilevel FMM. */
#define BEM_METHOD_BEM 0
#define BEM_METHOD_SLFMM 1
#define BEM_METHOD_MLFMM 4

/* Largest distance between two of the mesh's nodes (the diameter D of the
 * scatterer in the switching rules).  xyz: host double[n_nodes][3].  Host
 * only, O(n_nodes^2) over the host's threads. */
bem_status bem_mesh_diameter(int64_t n_nodes, const double* xyz, double* diameter);

/* The method the paper's safeguards turn a requested method into, for a mesh
 * of n_tri elements and diameter D at wavenumber k (lambda = 2 pi / k), the
 * rules applied in this order:
 *   requested BEM and n_tri > 20000            -> SLFMM
 *   BEM or SLFMM (after the above), n_tri > 50000 -> MLFMM
 *   an FMM and lambda >= 80 D                   -> BEM
 *   MLFMM and lambda > D                        -> SLFMM
 * *method receives BEM_METHOD_*.  Host only.  BEM_E_ARG for an unknown
 * method or a non-positive size, diameter or wavenumber. */
bem_status bem_auto_method(int32_t requested, int64_t n_tri, double diameter, double k, int32_t* method);

const char* bem_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BEMFMM_H */
