// FP64 sine and cosine for |x| < 2^20 by Cody & Waite reduction modulo pi/2
// (pi/2 split into three parts, the first two with 20 significant bits so that
// n*C1 and n*C2 are exact) and the Taylor series of sin and cos on
// [-pi/4, pi/4] truncated after the 1/17! and 1/16! terms (truncation error
// < 5e-17).  For the phases of the FMM setup kernels, which stay far below the
// range limit.
#pragma once

#include <hip/hip_runtime.h>

namespace bem {

__device__ inline void sincos_cw_lit(double x, double* s, double* c) {
  const double n = rint(x * 0.6366197723675814);
  double y = fma(-n, 1.5707950592041016, x);
  y = fma(-n, 1.2675900507019833e-06, y);
  y = fma(-n, 7.443547480486623e-13, y);
  const double z = y * y;
  double ps = 1.0 / 355687428096000.0;
  ps = fma(ps, z, -1.0 / 1307674368000.0);
  ps = fma(ps, z, 1.0 / 6227020800.0);
  ps = fma(ps, z, -1.0 / 39916800.0);
  ps = fma(ps, z, 1.0 / 362880.0);
  ps = fma(ps, z, -1.0 / 5040.0);
  ps = fma(ps, z, 1.0 / 120.0);
  ps = fma(ps, z, -1.0 / 6.0);
  const double sy = fma(y * z, ps, y);
  double pc = 1.0 / 20922789888000.0;
  pc = fma(pc, z, -1.0 / 87178291200.0);
  pc = fma(pc, z, 1.0 / 479001600.0);
  pc = fma(pc, z, -1.0 / 3628800.0);
  pc = fma(pc, z, 1.0 / 40320.0);
  pc = fma(pc, z, -1.0 / 720.0);
  pc = fma(pc, z, 1.0 / 24.0);
  pc = fma(pc, z, -0.5);
  const double cy = fma(z, pc, 1.0);
  const int q = ((int)n) & 3;
  const double a = (q & 1) ? cy : sy;
  const double b = (q & 1) ? sy : cy;
  *s = (q & 2) ? -a : a;
  *c = ((q + 1) & 2) ? -b : b;
}

}  // namespace bem
