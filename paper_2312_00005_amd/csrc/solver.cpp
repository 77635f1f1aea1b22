// Krylov driver: restarted GMRES with classical Gram-Schmidt applied twice,
// FP64 basis vectors and FP64 residuals (Sec. 3.2 uses CGS with a 1e-9
// tolerance and a 250-iteration cap; GMRES takes its place here), right
// preconditioned by the block-Jacobi inverse M (A M u = b, x = M u), so that
// its residual is the residual of the unpreconditioned system.  With the
// mixed precision option the inner solves run on the complex-FP32 operator
// inside an FP64 iterative-refinement loop: r = b - A x with the FP64
// operator, inner GMRES on A d = r, x += d.
#include <algorithm>
#include <complex>

#include "state.h"

namespace bem {

namespace {

using cd = std::complex<double>;

struct Work {
  int64_t N;
  int restart;
  int nblk;
};

// y = A x (tree order) for the Krylov loop: with use_graphs the kernel
// sequence of one application is captured once per (operator, precision,
// buffers, problem) on a private stream and replayed on s.
void apply_iter(bem_mesh* m, bem_op op, bem_precision prec, const double2* x, double2* y, hipStream_t s) {
  if (!m->opt.use_graphs) {
    apply_tree(m, op, prec, x, y, s);
    return;
  }
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
  BEM_HIP(hipGraphLaunch(G.exec, s));
}

double vec_norm(bem_mesh* m, const double2* v, const Work& W, hipStream_t s) {
  launch_multidot(W.N, 1, v, W.N, v, m->d_partial.p, W.nblk, s);
  launch_reduce_partials(1, W.nblk, m->d_partial.p, m->d_h.p, s);
  double2 h;
  BEM_HIP(hipMemcpyAsync(&h, m->d_h.p, sizeof(double2), hipMemcpyDeviceToHost, s));
  BEM_HIP(hipStreamSynchronize(s));
  return std::sqrt(std::max(0.0, h.x));
}

// One restarted GMRES solve of A x = b with operator precision prec.  x holds
// the initial guess (x_zero: treat it as zero).  Stops when the residual
// estimate falls below tol_abs, or after maxit iterations in total.
int gmres(bem_mesh* m, bem_op op, bem_precision prec, const double2* b, double2* x, bool x_zero, double tol_abs,
          int maxit, const Work& W, hipStream_t s, bool* converged) {
  const int64_t N = W.N;
  const int R = W.restart;
  double2* V = m->d_V.p;
  double2* w = m->d_w.p;
  double2* r = m->d_r.p;
  double2* dh = m->d_h.p;  // [0, R+1): h1, [R+1, 2R+2): h2, [2R+2]: norm
  int iters = 0;
  *converged = false;
  std::vector<cd> H((R + 1) * R), g(R + 1), cs(R), sn(R);
  std::vector<double2> hh(2 * (R + 1) + 1);
  for (;;) {
    if (x_zero) {
      BEM_HIP(hipMemcpyAsync(r, b, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
      BEM_HIP(hipMemsetAsync(x, 0, N * sizeof(double2), s));
      x_zero = false;
    } else {
      apply_tree(m, op, prec, x, w, s);
      launch_axpby(N, make_double2(1, 0), b, make_double2(-1, 0), w, r, s);
    }
    double beta = vec_norm(m, r, W, s);
    if (beta <= tol_abs) {
      *converged = true;
      return iters;
    }
    if (iters >= maxit) return iters;
    launch_scale_copy(N, r, make_double2(1.0 / beta, 0.0), V, s);
    std::fill(g.begin(), g.end(), cd(0));
    g[0] = beta;
    int jend = -1;
    bool done = false;
    for (int j = 0; j < R; ++j) {
      if (m->precond_ready) {
        precondition(m, op, V + (int64_t)j * N, m->d_z.p, s);
      } else {
        BEM_HIP(hipMemcpyAsync(m->d_z.p, V + (int64_t)j * N, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
      }
      apply_iter(m, op, prec, m->d_z.p, w, s);
      ++iters;
      // classical Gram-Schmidt, twice
      launch_multidot(N, j + 1, V, N, w, m->d_partial.p, W.nblk, s);
      launch_reduce_partials(j + 1, W.nblk, m->d_partial.p, dh, s);
      launch_multiaxpy(N, j + 1, V, N, dh, -1.0, w, s);
      launch_multidot(N, j + 1, V, N, w, m->d_partial.p, W.nblk, s);
      launch_reduce_partials(j + 1, W.nblk, m->d_partial.p, dh + (R + 1), s);
      launch_multiaxpy(N, j + 1, V, N, dh + (R + 1), -1.0, w, s);
      launch_multidot(N, 1, w, N, w, m->d_partial.p, W.nblk, s);
      launch_reduce_partials(1, W.nblk, m->d_partial.p, dh + 2 * (R + 1), s);
      BEM_HIP(hipMemcpyAsync(hh.data(), dh, hh.size() * sizeof(double2), hipMemcpyDeviceToHost, s));
      BEM_HIP(hipStreamSynchronize(s));
      const double hn = std::sqrt(std::max(0.0, hh[2 * (R + 1)].x));
      for (int i = 0; i <= j; ++i) H[i * R + j] = cd(hh[i].x + hh[R + 1 + i].x, hh[i].y + hh[R + 1 + i].y);
      H[(j + 1) * R + j] = hn;
      if (hn > 0.0) launch_scale_copy(N, w, make_double2(1.0 / hn, 0.0), V + (int64_t)(j + 1) * N, s);
      // apply the previous rotations and build the new one
      for (int i = 0; i < j; ++i) {
        cd a = H[i * R + j], bb = H[(i + 1) * R + j];
        H[i * R + j] = std::conj(cs[i]) * a + std::conj(sn[i]) * bb;
        H[(i + 1) * R + j] = -sn[i] * a + cs[i] * bb;
      }
      cd a = H[j * R + j], bb = H[(j + 1) * R + j];
      double den = std::sqrt(std::norm(a) + std::norm(bb));
      if (den == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else {
        cs[j] = a / den;
        sn[j] = bb / den;
      }
      H[j * R + j] = std::conj(cs[j]) * a + std::conj(sn[j]) * bb;
      H[(j + 1) * R + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = std::conj(cs[j]) * g[j];
      jend = j;
      const double res = std::abs(g[j + 1]);
      if (res <= tol_abs || iters >= maxit || hn == 0.0) {
        done = true;
        break;
      }
    }
    // back substitution and update x += V y
    const int nj = jend + 1;
    std::vector<cd> y(nj);
    for (int i = nj - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int l = i + 1; l < nj; ++l) acc -= H[i * R + l] * y[l];
      y[i] = acc / H[i * R + i];
    }
    std::vector<double2> yh(nj);
    for (int i = 0; i < nj; ++i) yh[i] = make_double2(y[i].real(), y[i].imag());
    BEM_HIP(hipMemcpyAsync(dh, yh.data(), nj * sizeof(double2), hipMemcpyHostToDevice, s));
    if (m->precond_ready) {
      // x += M (V y)
      BEM_HIP(hipMemsetAsync(m->d_z.p, 0, N * sizeof(double2), s));
      launch_multiaxpy(N, nj, V, N, dh, 1.0, m->d_z.p, s);
      precondition(m, op, m->d_z.p, w, s);
      launch_axpby(N, make_double2(1, 0), x, make_double2(1, 0), w, x, s);
    } else {
      launch_multiaxpy(N, nj, V, N, dh, 1.0, x, s);
    }
    BEM_HIP(hipStreamSynchronize(s));
    if (done && iters >= maxit) {
      // recompute the true residual to decide
      apply_tree(m, op, prec, x, w, s);
      launch_axpby(N, make_double2(1, 0), b, make_double2(-1, 0), w, r, s);
      *converged = vec_norm(m, r, W, s) <= tol_abs;
      return iters;
    }
  }
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
    BEM_HIP(hipMemsetAsync(x, 0, N * sizeof(double2), s));
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

}  // namespace

SolveResult solve_tree(bem_mesh* m, const double2* b, double2* x, hipStream_t s, bem_op op) {
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
  auto krylov = m->opt.solver == 1 ? cgs : gmres;
  const double bnorm = vec_norm(m, b, W, s);
  if (bnorm == 0.0) {
    BEM_HIP(hipMemsetAsync(x, 0, N * sizeof(double2), s));
    out.converged = true;
    return out;
  }
  const double tol = m->opt.gmres_tol;
  if (m->opt.precision == BEM_PREC_FP64) {
    bool conv = false;
    out.iterations = krylov(m, op, BEM_PREC_FP64, b, x, true, tol * bnorm, m->opt.gmres_maxit, W, s, &conv);
  } else {
    // FP64 iterative refinement around the complex-FP32 operator; rr always
    // holds the FP64 residual of the current x, so it also gives the final
    // residual without another application
    BEM_HIP(hipMemsetAsync(x, 0, N * sizeof(double2), s));
    BEM_HIP(hipMemcpyAsync(m->d_tmp.p, b, N * sizeof(double2), hipMemcpyDeviceToDevice, s));
    double2* rr = m->d_tmp.p;
    double2* d = m->d_y.p;
    double rn = vec_norm(m, rr, W, s);
    for (int it = 0; it < std::max(1, m->opt.refine_maxit); ++it) {
      if (rn <= tol * bnorm) break;
      bool conv = false;
      out.iterations += krylov(m, op, BEM_PREC_MIXED, rr, d, true, m->opt.inner_tol * rn,
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
  // true FP64 residual (GMRES stops on its own estimate)
  apply_tree(m, op, BEM_PREC_FP64, x, m->d_w.p, s);
  launch_axpby(N, make_double2(1, 0), b, make_double2(-1, 0), m->d_w.p, m->d_r.p, s);
  out.rel_residual = vec_norm(m, m->d_r.p, W, s) / bnorm;
  out.converged = out.rel_residual <= tol * (1.0 + 1e-6);
  return out;
}

}  // namespace bem
