// Block-Jacobi preconditioner: each block (a leaf cluster's near-field
// interactions among its own elements, at most kMaxBlock of them) is inverted
// in LDS by Gauss-Jordan elimination with partial pivoting, one workgroup per
// block, in FP64; the apply is a block-diagonal matrix-vector product.
#include "device.h"

namespace bem {

namespace {

constexpr int kLd = kMaxBlock + 1;  // padded LDS row

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline double2 cinv(double2 a) {
  const double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}

__global__ __launch_bounds__(256) void k_block_invert(BlockArgs B, const double2* __restrict__ A,
                                                      double2* __restrict__ out, int32_t* __restrict__ singular) {
  __shared__ double2 a[kMaxBlock * kLd];
  __shared__ double2 f[kMaxBlock];
  __shared__ int piv[kMaxBlock];
  __shared__ int prow;
  __shared__ int bad;
  const int64_t blk = blockIdx.x;
  const int n = B.n[blk];
  const int64_t off = B.off[blk];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < n * n; idx += 256) a[(idx % n) * kLd + idx / n] = A[off + idx];
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    // pivot: the largest |a[i][k]|, i >= k (first index on ties)
    if (tid < 64) {
      double v = -1.0;
      int idx = tid;
      if (tid >= k && tid < n) {
        const double2 z = a[tid * kLd + k];
        v = z.x * z.x + z.y * z.y;
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const double ov = __shfl_xor(v, o, 64);
        const int oi = __shfl_xor(idx, o, 64);
        if (ov > v || (ov == v && oi < idx)) {
          v = ov;
          idx = oi;
        }
      }
      if (tid == 0) {
        prow = idx;
        if (!(v > 0.0)) bad = 1;
      }
    }
    __syncthreads();
    if (bad) break;
    const int p = prow;
    if (p != k) {
      for (int c = tid; c < n; c += 256) {
        const double2 t = a[k * kLd + c];
        a[k * kLd + c] = a[p * kLd + c];
        a[p * kLd + c] = t;
      }
    }
    if (tid == 0) piv[k] = p;
    __syncthreads();
    const double2 inv = cinv(a[k * kLd + k]);
    for (int i = tid; i < n; i += 256) f[i] = a[i * kLd + k];
    __syncthreads();
    for (int c = tid; c < n; c += 256) a[k * kLd + c] = c == k ? inv : cmul(a[k * kLd + c], inv);
    __syncthreads();
    for (int idx = tid; idx < n * n; idx += 256) {
      const int i = idx / n, c = idx % n;
      if (i == k) continue;
      const double2 fi = f[i];
      if (c == k) {
        const double2 q = cmul(fi, inv);
        a[i * kLd + k] = make_double2(-q.x, -q.y);
      } else {
        const double2 q = cmul(fi, a[k * kLd + c]);
        a[i * kLd + c] = make_double2(a[i * kLd + c].x - q.x, a[i * kLd + c].y - q.y);
      }
    }
    __syncthreads();
  }
  if (bad) {
    // no usable pivot: fall back to the inverse of the diagonal
    for (int idx = tid; idx < n * n; idx += 256) {
      const int r = idx % n, c = idx / n;
      double2 v = make_double2(0.0, 0.0);
      if (r == c) {
        const double2 d = A[off + idx];
        v = (d.x != 0.0 || d.y != 0.0) ? cinv(d) : make_double2(1.0, 0.0);
      }
      out[off + idx] = v;
    }
    if (tid == 0) singular[blk] = 1;
    return;
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = n - 1; k >= 0; --k) {
    const int p = piv[k];
    if (p != k) {
      for (int r = tid; r < n; r += 256) {
        const double2 t = a[r * kLd + k];
        a[r * kLd + k] = a[r * kLd + p];
        a[r * kLd + p] = t;
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < n * n; idx += 256) out[off + idx] = a[(idx % n) * kLd + idx / n];
  if (tid == 0) singular[blk] = 0;
}

__global__ __launch_bounds__(256) void k_block_apply(int64_t N, BlockArgs B, const double2* __restrict__ inv,
                                                     int conj_t, const double2* __restrict__ x,
                                                     double2* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N) return;
  const int blk = B.elem_blk[t];
  const int64_t b0 = B.beg[blk];
  const int n = B.n[blk];
  const int64_t off = B.off[blk];
  const int il = (int)(t - b0);
  double ar = 0.0, ai = 0.0;
  if (!conj_t) {
    for (int jl = 0; jl < n; ++jl) {
      const double2 mv = inv[off + (int64_t)jl * n + il];
      const double2 xv = x[b0 + jl];
      ar += mv.x * xv.x - mv.y * xv.y;
      ai += mv.x * xv.y + mv.y * xv.x;
    }
  } else {
    for (int jl = 0; jl < n; ++jl) {
      const double2 mv = inv[off + (int64_t)il * n + jl];
      const double2 xv = x[b0 + jl];
      ar += mv.x * xv.x + mv.y * xv.y;
      ai += mv.x * xv.y - mv.y * xv.x;
    }
  }
  y[t] = make_double2(ar, ai);
}

}  // namespace

void launch_block_invert(const BlockArgs& B, const double2* a, double2* inv, int32_t* singular, hipStream_t s) {
  if (B.nblk <= 0) return;
  hipLaunchKernelGGL(k_block_invert, dim3((unsigned)B.nblk), dim3(256), 0, s, B, a, inv, singular);
}

void launch_block_apply(int64_t N, const BlockArgs& B, const double2* inv, bool conj_t, const double2* x,
                        double2* y, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(k_block_apply, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, B, inv,
                     conj_t ? 1 : 0, x, y);
}

}  // namespace bem
