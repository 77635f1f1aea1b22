// Krylov driver: restarted GMRES with classical Gram-Schmidt applied twice,
// FP64 basis vectors and FP64 residuals (Sec. 3.2 uses CGS with a 1e-9
// tolerance and a 250-iteration cap; GMRES takes its place here), right
// preconditioned by the block-Jacobi inverse M (A M u = b, x = M u), so that
// its residual is the residual of the unpreconditioned system.  With the
// mixed precision option the inner solves run on the complex-FP32 operator
// inside an FP64 iterative-refinement loop: r = b - A x with the FP64
// operator, inner GMRES on A d = r, x += d.  An inner solve reduces its
// residual by inner_tol, but never below half the outer target: the step
// that only has to close a small gap to the target stops after a few
// iterations instead of running the full inner reduction.
#include <algorithm>
#include <complex>
#include <memory>

#include "state.h"

namespace bem {

namespace {

using cd = std::complex<double>;

// absolute residual target of the inner solve of one refinement step: rn the
// current FP64 residual norm, target the outer one (tol |b|)
inline double inner_target(const bem_options& o, double rn, double target) {
  return std::max(o.inner_tol * rn, 0.5 * target);
}

struct Work {
  int64_t N;
  int restart;
  int nblk;
};

// Capture (once per operator, precision, buffers and problem) the kernel
// sequence of one application y = A x on a private stream, unless it is
// captured already.
void ensure_graph(bem_mesh* m, bem_op op, bem_precision prec, const double2* x, double2* y, hipStream_t s) {
  auto& G = m->graphs[op == BEM_OP_AH ? 1 : 0][prec == BEM_PREC_MIXED ? 1 : 0];
  if (!G.exec || G.stamp != m->problem_stamp || G.in != x || G.out != y) {
    if (G.exec) {
      BEM_HIP(hipGraphExecDestroy(G.exec));
      G.exec = nullptr;
    }
    if (op == BEM_OP_AH) ensure_transposed_plan(m, s);
    if (!m->cap_stream) BEM_HIP(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    BEM_HIP(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal));
    m->capturing = true;
    try {
      apply_tree(m, op, prec, x, y, m->cap_stream);
    } catch (...) {
      m->capturing = false;
      (void)hipStreamEndCapture(m->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    m->capturing = false;
    BEM_HIP(hipStreamEndCapture(m->cap_stream, &g));
    const hipError_t e = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    BEM_HIP(e);
    G.stamp = m->problem_stamp;
    G.in = x;
    G.out = y;
  }
}

// y = A x (tree order) for the Krylov loop: with use_graphs the captured
// application is replayed on s.
void apply_iter(bem_mesh* m, bem_op op, bem_precision prec, const double2* x, double2* y, hipStream_t s) {
  if (!m->opt.use_graphs) {
    apply_tree(m, op, prec, x, y, s);
    return;
  }
  ensure_graph(m, op, prec, x, y, s);
  BEM_HIP(hipGraphLaunch(m->graphs[op == BEM_OP_AH ? 1 : 0][prec == BEM_PREC_MIXED ? 1 : 0].exec, s));
}

double vec_norm(bem_mesh* m, const double2* v, const Work& W, hipStream_t s) {
  launch_multidot(W.N, 1, v, W.N, v, m->d_partial.p, W.nblk, s);
  launch_reduce_partials(1, W.nblk, m->d_partial.p, m->d_h.p, s);
  double2 h;
  BEM_HIP(hipMemcpyAsync(&h, m->d_h.p, sizeof(double2), hipMemcpyDeviceToHost, s));
  BEM_HIP(hipStreamSynchronize(s));
  return std::sqrt(std::max(0.0, h.x));
}

// Conjugate gradient squared (the paper's iterative solver, Sec. 3.2), right
// preconditioned like GMRES: on A M y = b with x = M y,
//   r = b - A x, rh = r, u = p = r, rho = (rh, r);
//   v = A M p, alpha = rho / (rh, v), q = u - alpha v, w = u + q,
//   x += alpha M w, r -= alpha A M w, rho' = (rh, r), beta = rho'/rho,
//   u = r + beta q, p = u + beta (q + beta p).
// Two operator applications per iteration; stops on the residual norm, after
// maxit iterations, or on a breakdown (rho or (rh, v) zero).
int cgs(bem_mesh* m, bem_op op, bem_precision prec, const double2* b, double2* x, bool x_zero, double tol_abs,
        int maxit, const Work& W, hipStream_t s, bool* converged) {
  const int64_t N = W.N;
  double2* V = m->d_V.p;
  double2* rh = V;             // rh and r adjacent: one pass gives (rh, r) and (r, r)
  double2* r = V + N;
  double2* u = V + 2 * N;
  double2* p = V + 3 * N;
  double2* q = V + 4 * N;
  double2* v = V + 5 * N;
  double2* w = V + 6 * N;
  double2* z = m->d_z.p;
  double2* dh = m->d_h.p;
  *converged = false;
  auto dots = [&](int nv, const double2* vecs, const double2* with, double2* out) {
    launch_multidot(N, nv, vecs, N, with, m->d_partial.p, W.nblk, s);
    launch_reduce_partials(nv, W.nblk, m->d_partial.p, dh, s);
    BEM_HIP(hipMemcpyAsync(out, dh, nv * sizeof(double2), hipMemcpyDeviceToHost, s));
    BEM_HIP(hipStreamSynchronize(s));
  };
  auto apply_m = [&](const double2* in, double2* out) {  // out = A M in
    precondition(m, op, in, z, s);
    apply_iter(m, op, prec, z, out, s);
  };
  if (x_zero) {
    launch_zero(N, x, s);
    BEM_HIP(hipMemcpyAsync(r, b, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
  } else {
    apply_tree(m, op, prec, x, w, s);
    launch_axpby(N, make_double2(1, 0), b, make_double2(-1, 0), w, r, s);
  }
  BEM_HIP(hipMemcpyAsync(rh, r, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
  BEM_HIP(hipMemcpyAsync(u, r, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
  BEM_HIP(hipMemcpyAsync(p, r, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
  double2 hr[2];
  dots(2, rh, r, hr);
  cd rho(hr[0].x, hr[0].y);
  if (std::sqrt(std::max(0.0, hr[1].x)) <= tol_abs) {
    *converged = true;
    return 0;
  }
  int it = 0;
  while (it < maxit) {
    ++it;
    apply_m(p, v);
    double2 sv;
    dots(1, rh, v, &sv);
    const cd sigma(sv.x, sv.y);
    if (sigma == cd(0.0) || rho == cd(0.0)) break;
    const cd alpha = rho / sigma;
    const double2 a2 = make_double2(alpha.real(), alpha.imag());
    // q = u - alpha v, w = u + q
    launch_axpby(N, make_double2(1, 0), u, make_double2(-a2.x, -a2.y), v, q, s);
    launch_axpby(N, make_double2(1, 0), u, make_double2(1, 0), q, w, s);
    // x += alpha M w; r -= alpha A M w  (v is free again: it holds A M w)
    precondition(m, op, w, z, s);
    launch_axpby(N, make_double2(1, 0), x, a2, z, x, s);
    apply_iter(m, op, prec, z, v, s);
    launch_axpby(N, make_double2(1, 0), r, make_double2(-a2.x, -a2.y), v, r, s);
    dots(2, rh, r, hr);
    if (std::sqrt(std::max(0.0, hr[1].x)) <= tol_abs) {
      *converged = true;
      break;
    }
    const cd rho_new(hr[0].x, hr[0].y);
    const cd beta = rho_new / rho;
    rho = rho_new;
    const double2 b2 = make_double2(beta.real(), beta.imag());
    // u = r + beta q; p = u + beta (q + beta p)
    launch_axpby(N, make_double2(1, 0), r, b2, q, u, s);
    launch_axpby(N, make_double2(1, 0), q, b2, p, p, s);
    launch_axpby(N, make_double2(1, 0), u, b2, p, p, s);
  }
  BEM_HIP(hipStreamSynchronize(s));
  return it;
}

// One solve of op(A) x = b by restarted GMRES (with the FP64 refinement loop
// around it in the mixed path), written as a sequence of phases so that the
// solves of several independent systems can advance in lock-step: each phase
// enqueues its device work on the system's stream and ends with one
// asynchronous copy of the scalars the host needs (a norm, or the
// Gram-Schmidt coefficients of one Arnoldi step) into pinned host memory;
// consume() reads them once they have landed, does the host part (Givens
// rotations, convergence tests, back substitution) and picks the next phase.
// While one system's scalars travel, the other systems' kernels keep the
// device busy.  The arithmetic and its order are those of the plain loop:
//   restart: r = b - A x (or r = b when x starts at zero), beta = |r|,
//            V_0 = r / beta;
//   step j:  w = A M V_j, classical Gram-Schmidt twice against V_0..V_j,
//            V_{j+1} = w / |w|, Givens rotation of the new Hessenberg column;
//   end of a cycle (converged estimate, breakdown, cap, or restart length):
//            x += M V y from the triangular solve, then a restart, which also
//            recomputes the true residual that decides convergence.
class SolveTask {
 public:
  SolveTask(bem_mesh* m, const double2* b, double2* x, hipStream_t s, bem_op op)
      : m_(m), b_(b), x_(x), s_(s), op_(op) {
    const int64_t N = m->N;
    W_ = Work{N, std::max(1, std::min(m->opt.gmres_restart, 200)), multidot_blocks(N)};
    const int R = W_.restart;
    m->d_V.alloc((size_t)std::max(R + 1, 8) * N);
    m->d_w.alloc(N);
    m->d_r.alloc(N);
    m->d_tmp.alloc(N);
    m->d_z.alloc(N);
    m->d_partial.alloc((size_t)(R + 1) * W_.nblk + 8);
    m->d_h.alloc(2 * (R + 1) + 8);
    H_.assign((size_t)(R + 1) * R, cd(0));
    g_.assign(R + 1, cd(0));
    cs_.assign(R, cd(0));
    sn_.assign(R, cd(0));
    nhost_ = 3 * (R + 1) + 8;
    BEM_HIP(hipHostMalloc((void**)&host_, nhost_ * sizeof(double2), hipHostMallocDefault));
    if (hipEventCreateWithFlags(&ev_, hipEventDisableTiming) != hipSuccess) {
      (void)hipHostFree(host_);
      throw Error(BEM_E_HIP, "hipEventCreateWithFlags failed");
    }
    mixed_ = m->opt.precision == BEM_PREC_MIXED;
    tol_ = m->opt.gmres_tol;
  }
  ~SolveTask() {
    if (ev_) (void)hipEventSynchronize(ev_);
    if (ev_) (void)hipEventDestroy(ev_);
    if (host_) (void)hipHostFree(host_);
  }
  SolveTask(const SolveTask&) = delete;
  SolveTask& operator=(const SolveTask&) = delete;

  bool done() const { return phase_ == kDone; }
  const SolveResult& result() const { return out_; }

  // Captured applications of the inner operator, made before the lock-step
  // loop so that no capture overlaps another system's work.
  void prepare() {
    if (m_->opt.use_graphs)
      ensure_graph(m_, op_, mixed_ ? BEM_PREC_MIXED : BEM_PREC_FP64, m_->d_z.p, m_->d_w.p, s_);
  }

  void enqueue() {
    const int64_t N = W_.N;
    switch (phase_) {
      case kNormB:
        norm_async(b_);
        break;
      case kGmStart:
        if (gx_zero_) {
          BEM_HIP(hipMemcpyAsync(m_->d_r.p, grhs_, N * sizeof(double2), hipMemcpyDeviceToDevice, s_));
          launch_zero(N, gsol_, s_);
        } else {
          apply_tree(m_, op_, gprec_, gsol_, m_->d_w.p, s_);
          launch_axpby(N, make_double2(1, 0), grhs_, make_double2(-1, 0), m_->d_w.p, m_->d_r.p, s_);
        }
        norm_async(m_->d_r.p);
        break;
      case kGmIter:
        arnoldi_async();
        break;
      case kGmTrueResid:
        apply_tree(m_, op_, gprec_, gsol_, m_->d_w.p, s_);
        launch_axpby(N, make_double2(1, 0), grhs_, make_double2(-1, 0), m_->d_w.p, m_->d_r.p, s_);
        norm_async(m_->d_r.p);
        break;
      case kFinal:
        // true FP64 residual (GMRES stops on its own estimate)
        apply_tree(m_, op_, BEM_PREC_FP64, x_, m_->d_w.p, s_);
        launch_axpby(N, make_double2(1, 0), b_, make_double2(-1, 0), m_->d_w.p, m_->d_r.p, s_);
        norm_async(m_->d_r.p);
        break;
      case kRefine:
        // x += d; rr = b - A x with the FP64 operator
        launch_axpby(N, make_double2(1, 0), x_, make_double2(1, 0), m_->d_y.p, x_, s_);
        apply_tree(m_, op_, BEM_PREC_FP64, x_, m_->d_w.p, s_);
        launch_axpby(N, make_double2(1, 0), b_, make_double2(-1, 0), m_->d_w.p, m_->d_tmp.p, s_);
        norm_async(m_->d_tmp.p);
        break;
      case kDone:
        return;
    }
    BEM_HIP(hipEventRecord(ev_, s_));
  }

  void wait() {
    if (phase_ != kDone) BEM_HIP(hipEventSynchronize(ev_));
  }

  void consume() {
    switch (phase_) {
      case kNormB: {
        bnorm_ = norm_value();
        if (bnorm_ == 0.0) {
          launch_zero(W_.N, x_, s_);
          out_.converged = true;
          finish();
          return;
        }
        if (!mixed_) {
          begin_gmres(b_, x_, BEM_PREC_FP64, tol_ * bnorm_, kFinal);
        } else {
          // FP64 iterative refinement around the complex-FP32 operator; rr
          // (d_tmp) always holds the FP64 residual of the current x
          launch_zero(W_.N, x_, s_);
          BEM_HIP(hipMemcpyAsync(m_->d_tmp.p, b_, W_.N * sizeof(double2), hipMemcpyDeviceToDevice, s_));
          rn_ = bnorm_;
          refine_it_ = 0;
          next_refinement();
        }
        return;
      }
      case kGmStart: {
        const double beta = norm_value();
        gx_zero_ = false;
        if (beta <= gtol_) {
          gconv_ = true;
          end_gmres();
          return;
        }
        if (giters_ >= m_->opt.gmres_maxit) {
          end_gmres();
          return;
        }
        launch_scale_copy(W_.N, m_->d_r.p, make_double2(1.0 / beta, 0.0), m_->d_V.p, s_);
        std::fill(g_.begin(), g_.end(), cd(0));
        g_[0] = beta;
        j_ = 0;
        phase_ = kGmIter;
        return;
      }
      case kGmIter:
        givens_step();
        return;
      case kGmTrueResid:
        gconv_ = norm_value() <= gtol_;
        end_gmres();
        return;
      case kFinal:
        out_.rel_residual = norm_value() / bnorm_;
        out_.converged = out_.rel_residual <= tol_ * (1.0 + 1e-6);
        finish();
        return;
      case kRefine:
        rn_ = norm_value();
        ++out_.refinements;
        ++refine_it_;
        if (out_.iterations >= m_->opt.gmres_maxit || refine_it_ >= std::max(1, m_->opt.refine_maxit)) {
          finish_refinement();
          return;
        }
        next_refinement();
        return;
      case kDone:
        return;
    }
  }

 private:
  enum Phase { kNormB, kGmStart, kGmIter, kGmTrueResid, kFinal, kRefine, kDone };

  double2* dh() const { return m_->d_h.p; }  // [0, R+1): h1, [R+1, 2R+2): h2, [2R+2]: norm

  void norm_async(const double2* v) {
    launch_multidot(W_.N, 1, v, W_.N, v, m_->d_partial.p, W_.nblk, s_);
    launch_reduce_partials(1, W_.nblk, m_->d_partial.p, dh(), s_);
    BEM_HIP(hipMemcpyAsync(host_, dh(), sizeof(double2), hipMemcpyDeviceToHost, s_));
  }
  double norm_value() const { return std::sqrt(std::max(0.0, host_[0].x)); }

  void arnoldi_async() {
    const int64_t N = W_.N;
    const int R = W_.restart;
    double2* V = m_->d_V.p;
    double2* w = m_->d_w.p;
    const int j = j_;
    if (m_->precond_ready) {
      precondition(m_, op_, V + (int64_t)j * N, m_->d_z.p, s_);
    } else {
      BEM_HIP(hipMemcpyAsync(m_->d_z.p, V + (int64_t)j * N, N * sizeof(double2), hipMemcpyDeviceToDevice, s_));
    }
    apply_iter(m_, op_, gprec_, m_->d_z.p, w, s_);
    // classical Gram-Schmidt, twice
    launch_multidot(N, j + 1, V, N, w, m_->d_partial.p, W_.nblk, s_);
    launch_reduce_partials(j + 1, W_.nblk, m_->d_partial.p, dh(), s_);
    launch_multiaxpy(N, j + 1, V, N, dh(), -1.0, w, s_);
    launch_multidot(N, j + 1, V, N, w, m_->d_partial.p, W_.nblk, s_);
    launch_reduce_partials(j + 1, W_.nblk, m_->d_partial.p, dh() + (R + 1), s_);
    launch_multiaxpy(N, j + 1, V, N, dh() + (R + 1), -1.0, w, s_);
    launch_multidot(N, 1, w, N, w, m_->d_partial.p, W_.nblk, s_);
    launch_reduce_partials(1, W_.nblk, m_->d_partial.p, dh() + 2 * (R + 1), s_);
    BEM_HIP(hipMemcpyAsync(host_, dh(), (2 * (R + 1) + 1) * sizeof(double2), hipMemcpyDeviceToHost, s_));
  }

  void givens_step() {
    const int64_t N = W_.N;
    const int R = W_.restart;
    const int j = j_;
    const double2* hh = host_;
    ++giters_;
    const double hn = std::sqrt(std::max(0.0, hh[2 * (R + 1)].x));
    for (int i = 0; i <= j; ++i) H_[i * R + j] = cd(hh[i].x + hh[R + 1 + i].x, hh[i].y + hh[R + 1 + i].y);
    H_[(j + 1) * R + j] = hn;
    if (hn > 0.0)
      launch_scale_copy(N, m_->d_w.p, make_double2(1.0 / hn, 0.0), m_->d_V.p + (int64_t)(j + 1) * N, s_);
    // apply the previous rotations and build the new one
    for (int i = 0; i < j; ++i) {
      const cd a = H_[i * R + j], bb = H_[(i + 1) * R + j];
      H_[i * R + j] = std::conj(cs_[i]) * a + std::conj(sn_[i]) * bb;
      H_[(i + 1) * R + j] = -sn_[i] * a + cs_[i] * bb;
    }
    const cd a = H_[j * R + j], bb = H_[(j + 1) * R + j];
    const double den = std::sqrt(std::norm(a) + std::norm(bb));
    if (den == 0.0) {
      cs_[j] = 1.0;
      sn_[j] = 0.0;
    } else {
      cs_[j] = a / den;
      sn_[j] = bb / den;
    }
    H_[j * R + j] = std::conj(cs_[j]) * a + std::conj(sn_[j]) * bb;
    H_[(j + 1) * R + j] = 0.0;
    g_[j + 1] = -sn_[j] * g_[j];
    g_[j] = std::conj(cs_[j]) * g_[j];
    const double res = std::abs(g_[j + 1]);
    const bool stop = res <= gtol_ || giters_ >= m_->opt.gmres_maxit || hn == 0.0;
    if (!stop && j + 1 < R) {
      ++j_;
      return;  // next Arnoldi step
    }
    update_solution(j + 1);
    // at the cap the true residual decides; otherwise the restart recomputes
    // it (and stops there if it is small enough)
    phase_ = (stop && giters_ >= m_->opt.gmres_maxit) ? kGmTrueResid : kGmStart;
  }

  // x += M V y with y from the triangular system H y = g (nj columns)
  void update_solution(int nj) {
    const int64_t N = W_.N;
    const int R = W_.restart;
    std::vector<cd> y(nj);
    for (int i = nj - 1; i >= 0; --i) {
      cd acc = g_[i];
      for (int l = i + 1; l < nj; ++l) acc -= H_[i * R + l] * y[l];
      y[i] = acc / H_[i * R + i];
    }
    // the y slot of the pinned buffer is rewritten only after at least one
    // more event wait, so the upload below has finished by then
    double2* yh = host_ + 2 * (R + 1) + 4;
    for (int i = 0; i < nj; ++i) yh[i] = make_double2(y[i].real(), y[i].imag());
    BEM_HIP(hipMemcpyAsync(dh(), yh, nj * sizeof(double2), hipMemcpyHostToDevice, s_));
    double2* V = m_->d_V.p;
    if (m_->precond_ready) {
      launch_zero(N, m_->d_z.p, s_);
      launch_multiaxpy(N, nj, V, N, dh(), 1.0, m_->d_z.p, s_);
      precondition(m_, op_, m_->d_z.p, m_->d_w.p, s_);
      launch_axpby(N, make_double2(1, 0), gsol_, make_double2(1, 0), m_->d_w.p, gsol_, s_);
    } else {
      launch_multiaxpy(N, nj, V, N, dh(), 1.0, gsol_, s_);
    }
  }

  void begin_gmres(const double2* rhs, double2* sol, bem_precision prec, double tol_abs, Phase after) {
    grhs_ = rhs;
    gsol_ = sol;
    gprec_ = prec;
    gtol_ = tol_abs;
    gx_zero_ = true;
    gconv_ = false;
    giters_ = 0;
    after_ = after;
    phase_ = kGmStart;
  }

  void end_gmres() {
    out_.iterations += giters_;
    phase_ = after_;
  }

  void next_refinement() {
    if (rn_ <= tol_ * bnorm_) {
      finish_refinement();
      return;
    }
    begin_gmres(m_->d_tmp.p, m_->d_y.p, BEM_PREC_MIXED, inner_target(m_->opt, rn_, tol_ * bnorm_), kRefine);
  }

  void finish_refinement() {
    out_.rel_residual = rn_ / bnorm_;
    out_.converged = out_.rel_residual <= tol_ * (1.0 + 1e-6);
    finish();
  }

  void finish() { phase_ = kDone; }

  bem_mesh* m_;
  const double2* b_;
  double2* x_;
  hipStream_t s_;
  bem_op op_;
  Work W_{};
  bool mixed_ = false;
  double tol_ = 0.0, bnorm_ = 0.0, rn_ = 0.0;
  int refine_it_ = 0;
  Phase phase_ = kNormB, after_ = kDone;
  // the GMRES run in progress
  const double2* grhs_ = nullptr;
  double2* gsol_ = nullptr;
  bem_precision gprec_ = BEM_PREC_FP64;
  double gtol_ = 0.0;
  bool gx_zero_ = true, gconv_ = false;
  int giters_ = 0, j_ = 0;
  std::vector<cd> H_, g_, cs_, sn_;
  double2* host_ = nullptr;
  size_t nhost_ = 0;
  hipEvent_t ev_ = nullptr;
  SolveResult out_;
};

// CGS (the paper's solver) runs its systems one after another.
SolveResult solve_tree_cgs(bem_mesh* m, const double2* b, double2* x, hipStream_t s, bem_op op) {
  const int64_t N = m->N;
  Work W{N, std::max(1, std::min(m->opt.gmres_restart, 200)), multidot_blocks(N)};
  m->d_V.alloc((size_t)std::max(W.restart + 1, 8) * N);
  m->d_w.alloc(N);
  m->d_r.alloc(N);
  m->d_tmp.alloc(N);
  m->d_z.alloc(N);
  m->d_partial.alloc((size_t)(W.restart + 1) * W.nblk + 8);
  m->d_h.alloc(2 * (W.restart + 1) + 8);
  SolveResult out;
  const double bnorm = vec_norm(m, b, W, s);
  if (bnorm == 0.0) {
    launch_zero(N, x, s);
    out.converged = true;
    return out;
  }
  const double tol = m->opt.gmres_tol;
  if (m->opt.precision == BEM_PREC_FP64) {
    bool conv = false;
    out.iterations = cgs(m, op, BEM_PREC_FP64, b, x, true, tol * bnorm, m->opt.gmres_maxit, W, s, &conv);
  } else {
    launch_zero(N, x, s);
    BEM_HIP(hipMemcpyAsync(m->d_tmp.p, b, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
    double2* rr = m->d_tmp.p;
    double2* d = m->d_y.p;
    double rn = vec_norm(m, rr, W, s);
    for (int it = 0; it < std::max(1, m->opt.refine_maxit); ++it) {
      if (rn <= tol * bnorm) break;
      bool conv = false;
      out.iterations += cgs(m, op, BEM_PREC_MIXED, rr, d, true, inner_target(m->opt, rn, tol * bnorm),
                            m->opt.gmres_maxit, W, s, &conv);
      ++out.refinements;
      launch_axpby(N, make_double2(1, 0), x, make_double2(1, 0), d, x, s);
      apply_tree(m, op, BEM_PREC_FP64, x, m->d_w.p, s);
      launch_axpby(N, make_double2(1, 0), b, make_double2(-1, 0), m->d_w.p, rr, s);
      rn = vec_norm(m, rr, W, s);
      if (out.iterations >= m->opt.gmres_maxit) break;
    }
    out.rel_residual = rn / bnorm;
    out.converged = out.rel_residual <= tol * (1.0 + 1e-6);
    return out;
  }
  apply_tree(m, op, BEM_PREC_FP64, x, m->d_w.p, s);
  launch_axpby(N, make_double2(1, 0), b, make_double2(-1, 0), m->d_w.p, m->d_r.p, s);
  out.rel_residual = vec_norm(m, m->d_r.p, W, s) / bnorm;
  out.converged = out.rel_residual <= tol * (1.0 + 1e-6);
  return out;
}

}  // namespace

std::vector<SolveResult> solve_tree_batch(const std::vector<BatchItem>& items, bem_op op) {
  std::vector<SolveResult> out(items.size());
  std::vector<std::unique_ptr<SolveTask>> tasks;
  std::vector<size_t> which;
  for (size_t i = 0; i < items.size(); ++i) {
    const BatchItem& it = items[i];
    if (it.m->opt.solver == 1) {
      out[i] = solve_tree_cgs(it.m, it.b, it.x, it.s, op);
      continue;
    }
    tasks.emplace_back(new SolveTask(it.m, it.b, it.x, it.s, op));
    which.push_back(i);
  }
  for (auto& t : tasks) t->prepare();
  for (;;) {
    bool any = false;
    for (auto& t : tasks)
      if (!t->done()) {
        t->enqueue();
        any = true;
      }
    if (!any) break;
    for (auto& t : tasks) {
      if (t->done()) continue;
      t->wait();
      t->consume();
    }
  }
  for (size_t q = 0; q < tasks.size(); ++q) out[which[q]] = tasks[q]->result();
  return out;
}

SolveResult solve_tree(bem_mesh* m, const double2* b, double2* x, hipStream_t s, bem_op op) {
  return solve_tree_batch({BatchItem{m, b, x, s}}, op)[0];
}

}  // namespace bem
