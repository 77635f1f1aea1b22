// FP64 vector kernels of the GMRES driver: block-partial dot products of a
// vector against several basis vectors (classical Gram-Schmidt, applied
// twice), their fixed-order reduction, multi-vector updates and scaling.
// Reductions are two-stage with a fixed summation order, so results do not
// depend on scheduling.
#include "device.h"

namespace bem {

namespace {

constexpr int kDotThreads = 256;
constexpr int kDotPerThread = 8;
constexpr int kDotChunk = kDotThreads * kDotPerThread;

// partial[i * nblk + b] = sum over block b's elements of conj(V_i[n]) w[n]
__global__ __launch_bounds__(kDotThreads) void k_multidot(int64_t N, int nv, const double2* __restrict__ V,
                                                          int64_t ldv, const double2* __restrict__ w,
                                                          double2* __restrict__ partial, int nblk) {
  __shared__ double sr[kDotThreads], si[kDotThreads];
  const int64_t base = (int64_t)blockIdx.x * kDotChunk;
  double2 wl[kDotPerThread];
#pragma unroll
  for (int q = 0; q < kDotPerThread; ++q) {
    const int64_t n = base + q * kDotThreads + threadIdx.x;
    wl[q] = n < N ? w[n] : make_double2(0.0, 0.0);
  }
  for (int i = 0; i < nv; ++i) {
    const double2* v = V + (int64_t)i * ldv;
    double ar = 0.0, ai = 0.0;
#pragma unroll
    for (int q = 0; q < kDotPerThread; ++q) {
      const int64_t n = base + q * kDotThreads + threadIdx.x;
      if (n < N) {
        const double2 a = v[n];
        ar += a.x * wl[q].x + a.y * wl[q].y;
        ai += a.x * wl[q].y - a.y * wl[q].x;
      }
    }
    sr[threadIdx.x] = ar;
    si[threadIdx.x] = ai;
    __syncthreads();
    for (int s = kDotThreads / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        sr[threadIdx.x] += sr[threadIdx.x + s];
        si[threadIdx.x] += si[threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)i * nblk + blockIdx.x] = make_double2(sr[0], si[0]);
    __syncthreads();
  }
}

__global__ void k_reduce_partials(int nv, int nblk, const double2* __restrict__ partial,
                                  double2* __restrict__ h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  double ar = 0.0, ai = 0.0;
  for (int b = 0; b < nblk; ++b) {
    const double2 p = partial[(int64_t)i * nblk + b];
    ar += p.x;
    ai += p.y;
  }
  h[i] = make_double2(ar, ai);
}

// w[n] += sign * sum_i h[i] V_i[n]
__global__ __launch_bounds__(256) void k_multiaxpy(int64_t N, int nv, const double2* __restrict__ V,
                                                   int64_t ldv, const double2* __restrict__ h, double sign,
                                                   double2* __restrict__ w) {
  __shared__ double2 hs[256];
  for (int i = threadIdx.x; i < nv && i < 256; i += blockDim.x) hs[i] = h[i];
  __syncthreads();
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double ar = 0.0, ai = 0.0;
  for (int i = 0; i < nv; ++i) {
    const double2 v = V[(int64_t)i * ldv + n];
    const double2 c = hs[i];
    ar += c.x * v.x - c.y * v.y;
    ai += c.x * v.y + c.y * v.x;
  }
  double2 o = w[n];
  w[n] = make_double2(o.x + sign * ar, o.y + sign * ai);
}

__global__ void k_scale_copy(int64_t N, const double2* __restrict__ w, double2 a, double2* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double2 v = w[n];
  out[n] = make_double2(a.x * v.x - a.y * v.y, a.x * v.y + a.y * v.x);
}

__global__ void k_fill_i64(int64_t n, int64_t value, int64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = value;
}

__global__ void k_zero(int64_t N, double2* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N) out[n] = make_double2(0.0, 0.0);
}

__global__ void k_axpby(int64_t N, double2 a, const double2* __restrict__ x, double2 b,
                        const double2* __restrict__ y, double2* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double2 u = x[n], v = y[n];
  out[n] = make_double2(a.x * u.x - a.y * u.y + b.x * v.x - b.y * v.y,
                        a.x * u.y + a.y * u.x + b.x * v.y + b.y * v.x);
}

}  // namespace

int multidot_blocks(int64_t N) { return (int)((N + kDotChunk - 1) / kDotChunk); }

void launch_multidot(int64_t N, int nv, const double2* V, int64_t ldv, const double2* w, double2* partial,
                     int nblk, hipStream_t s) {
  if (N <= 0 || nv <= 0) return;
  hipLaunchKernelGGL(k_multidot, dim3(nblk), dim3(kDotThreads), 0, s, N, nv, V, ldv, w, partial, nblk);
}

void launch_reduce_partials(int nv, int nblk, const double2* partial, double2* h, hipStream_t s) {
  if (nv <= 0) return;
  hipLaunchKernelGGL(k_reduce_partials, dim3((nv + 127) / 128), dim3(128), 0, s, nv, nblk, partial, h);
}

void launch_multiaxpy(int64_t N, int nv, const double2* V, int64_t ldv, const double2* h, double sign,
                      double2* w, hipStream_t s) {
  if (N <= 0 || nv <= 0) return;
  hipLaunchKernelGGL(k_multiaxpy, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, nv, V, ldv, h,
                     sign, w);
}

void launch_scale_copy(int64_t N, const double2* w, double2 alpha, double2* out, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, w, alpha, out);
}

void launch_fill_i64(int64_t n, int64_t value, int64_t* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, value, out);
}

void launch_zero(int64_t N, double2* out, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, out);
}

// Interior problem (tau = -1 in Eq. (SystemI)): with the exterior operator
// A = D + K (D = (1 - gamma c)/2 the jump term, K every integral term) the
// interior one is D - K = 2 D - A, so y = A x becomes y = -y + 2 D x.
// mode 0: A (2D = 1 - gamma c); 1: A^H (conj); 2: V = dA/dc, whose jump
// part is -gamma/2 (2D = -gamma); 3: V^H; 4: an integral part alone (-y).
__global__ void k_interior(int64_t N, int mode, double gre, double gim, const double2* __restrict__ cfac,
                           const double2* __restrict__ x, double2* __restrict__ y) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  const double2 v = y[n];
  if (mode == 4) {
    y[n] = make_double2(-v.x, -v.y);
    return;
  }
  double dr, di;  // 2 D_nn
  if (mode <= 1) {
    const double2 c = cfac ? cfac[n] : make_double2(0.0, 0.0);
    dr = 1.0 - (gre * c.x - gim * c.y);
    di = -(gre * c.y + gim * c.x);
  } else {
    dr = -gre;
    di = -gim;
  }
  if (mode == 1 || mode == 3) di = -di;
  const double2 u = x[n];
  y[n] = make_double2(-v.x + dr * u.x - di * u.y, -v.y + dr * u.y + di * u.x);
}

// out = x on the elements with mask m == keep, 0 elsewhere (m is 0 or 1)
__global__ void k_mask(int64_t N, const double* __restrict__ m, int keep, const double2* __restrict__ x,
                       double2* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  out[n] = (m[n] != 0.0) == (keep != 0) ? x[n] : make_double2(0.0, 0.0);
}

// y = y where m == 0, z where m == 1
__global__ void k_blend(int64_t N, const double* __restrict__ m, double2* __restrict__ y,
                        const double2* __restrict__ z) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  if (m[n] != 0.0) y[n] = z[n];
}

void launch_mask(int64_t N, const double* m, int keep, const double2* x, double2* out, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_mask, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, m, keep, x, out);
}

void launch_blend(int64_t N, const double* m, double2* y, const double2* z, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_blend, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, m, y, z);
}

void launch_interior(int64_t N, int mode, double gre, double gim, const double2* cfac, const double2* x,
                     double2* y, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_interior, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, mode, gre, gim, cfac, x, y);
}

void launch_axpby(int64_t N, double2 a, const double2* x, double2 b, const double2* y, double2* out,
                  hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, a, x, b, y, out);
}

}  // namespace bem
