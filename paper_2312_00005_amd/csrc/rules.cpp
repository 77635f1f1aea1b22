// One-dimensional Gauss rules on [0, 1], computed from the three-term
// recurrences of the orthogonal polynomials: every root is found by Newton's
// method with Maehly deflation, starting to the right of the largest remaining
// root (monotone convergence for polynomials with real simple roots).
//
//   Gauss-Legendre:          int_0^1 f(x) dx      (Legendre P_n on [-1, 1])
//   Gauss for weight xi:     int_0^1 xi f(xi) dxi (Jacobi P_n^(0,1) on [-1, 1])
//
// These are the 1-D factors of the regular conical triangle rule (Sec. 3.1.4),
// of the six-triangle Duffy rule (Sec. 3.1.1) and of the edge rule of the
// hypersingular self term (Sec. 3.1.2).
#include "common.h"

namespace bem {

namespace {

// Jacobi P_n^(a,b)(x) and its derivative by the three-term recurrence
// (Legendre for a = b = 0).
void jacobi_eval(int n, double a, double b, double x, double& p, double& dp) {
  double p0 = 1.0, d0 = 0.0;
  if (n == 0) { p = p0; dp = d0; return; }
  double p1 = 0.5 * ((a + b + 2.0) * x + a - b);
  double d1 = 0.5 * (a + b + 2.0);
  for (int k = 2; k <= n; ++k) {
    double s = 2.0 * k + a + b;
    double c1 = 2.0 * k * (k + a + b) * (s - 2.0);
    double c2 = (s - 1.0) * (s * (s - 2.0) * x + a * a - b * b);
    double c2d = (s - 1.0) * s * (s - 2.0);
    double c3 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * s;
    double p2 = (c2 * p1 - c3 * p0) / c1;
    double d2 = (c2 * d1 + c2d * p1 - c3 * d0) / c1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  p = p1;
  dp = d1;
}

void roots(int n, double a, double b, std::vector<double>& xr, std::vector<double>& dpr) {
  xr.assign(n, 0.0);
  dpr.assign(n, 0.0);
  double start = 1.0;
  for (int i = 0; i < n; ++i) {
    double x = start;
    for (int it = 0; it < 200; ++it) {
      double p, dp;
      jacobi_eval(n, a, b, x, p, dp);
      double s = 0.0;
      for (int j = 0; j < i; ++j) s += 1.0 / (x - xr[j]);
      double step = p / (dp - p * s);
      x -= step;
      if (std::fabs(step) < 1e-16 * (1.0 + std::fabs(x))) break;
    }
    // two polishing steps without deflation
    for (int it = 0; it < 2; ++it) {
      double p, dp;
      jacobi_eval(n, a, b, x, p, dp);
      x -= p / dp;
    }
    double p, dp;
    jacobi_eval(n, a, b, x, p, dp);
    xr[i] = x;
    dpr[i] = dp;
    start = x - 1e-12 * (1.0 + std::fabs(x));
  }
}

}  // namespace

void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> xr, dp;
  roots(n, 0.0, 0.0, xr, dp);
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    // ascending order on [0, 1]
    int s = n - 1 - i;
    double xi = xr[s];
    double wi = 2.0 / ((1.0 - xi * xi) * dp[s] * dp[s]);
    x[i] = 0.5 * (xi + 1.0);
    w[i] = 0.5 * wi;
  }
}

void gauss_jacobi_xi01(int n, std::vector<double>& x, std::vector<double>& w) {
  // weights of P_n^(0,1) on [-1, 1]: 4 / ((1 - x^2) P_n'(x)^2); mapping
  // xi = (1 + x)/2 turns int (1 + x) g dx into 4 int xi g dxi.
  std::vector<double> xr, dp;
  roots(n, 0.0, 1.0, xr, dp);
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    int s = n - 1 - i;
    double xi = xr[s];
    x[i] = 0.5 * (xi + 1.0);
    w[i] = 1.0 / ((1.0 - xi * xi) * dp[s] * dp[s]);
  }
}

}  // namespace bem
