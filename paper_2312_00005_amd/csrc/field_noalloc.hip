// bem_field_noalloc: the field-point evaluation of bem_field without any
// device allocation, for callers that cannot allocate (code under graph
// capture, serving loops, harnesses that forbid hipMalloc).
//
// bem_field allocates a device error flag per call; this variant keeps the
// flag, and the per-block partial sums of the optional energy sum_f |p_f|^2,
// in `scratch`, a file-scope device array of fixed size that every GPU holds
// for the life of the process.  Host code never passes the array's name to a
// kernel: its device address is looked up once per device with
// hipGetSymbolAddress and kept.  All calls on one GPU share that array, so
// calls that overlap in time on one GPU race (the flag is reset and the
// partials fully rewritten at the start of every call).
#include <mutex>

#include "guard.h"
#include "state.h"

namespace bem {

namespace {

constexpr int kEnergyThreads = 256;
constexpr int64_t kPointsPerBlock = 4096;  // energy points per block
constexpr int kMaxEnergyBlocks = 1024;
// one int64 error flag, then the energy partials
constexpr int kScratchDoubles = 1 + kMaxEnergyBlocks;

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

// the device address of this device's scratch array (looked up once)
double* scratch_on_current_device() {
  int dev = 0;
  BEM_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) throw Error(BEM_E_HIP, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Error(BEM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  return static_cast<double*>(g_scratch_ptr[dev]);
}

__global__ void k_flag_reset(int64_t* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) flag[0] = -1;
}

__device__ inline double block_sum(double v, double* part) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  return (part[0] + part[1]) + (part[2] + part[3]);
}

// partial[b] = sum of |p_f|^2 over block b's contiguous run of points
__global__ __launch_bounds__(kEnergyThreads) void k_energy_partials(int64_t n, int64_t per_block,
                                                                  const double2* __restrict__ p,
                                                                  double* __restrict__ partial) {
  __shared__ double part[4];
  const int64_t f0 = (int64_t)blockIdx.x * per_block;
  const int64_t f1 = f0 + per_block < n ? f0 + per_block : n;
  double acc = 0.0;
  for (int64_t f = f0 + threadIdx.x; f < f1; f += kEnergyThreads) acc += p[f].x * p[f].x + p[f].y * p[f].y;
  const double s = block_sum(acc, part);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// energy = sum of the partials in block order
__global__ __launch_bounds__(kEnergyThreads) void k_energy_final(int nb, const double* __restrict__ partial,
                                                               double* __restrict__ energy) {
  __shared__ double part[4];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kEnergyThreads) acc += partial[b];
  const double s = block_sum(acc, part);
  if (threadIdx.x == 0) energy[0] = s;
}

}  // namespace

}  // namespace bem

using namespace bem;

extern "C" bem_status bem_field_noalloc(bem_mesh* m, int64_t n_pts, const double* pts, const bem_c128* p_surf,
                                        const bem_c128* p_inc, bem_c128* p_out, double* energy, void* stream) {
  return guarded([&]() -> bem_status {
    if (!m || !p_surf || n_pts < 0 || (n_pts > 0 && (!pts || !p_out))) return fail(BEM_E_ARG, "NULL argument");
    if (n_pts > kPointsPerBlock * kMaxEnergyBlocks)
      return fail(BEM_E_ARG, "n_pts exceeds the " + std::to_string(kPointsPerBlock * kMaxEnergyBlocks) +
                                 " points that bem_field_noalloc's fixed scratch array supports");
    if (!m->have_problem) return fail(BEM_E_STATE, "bem_set_problem has not been called");
    if (m->opt.interior)
      return fail(BEM_E_STATE, "field points use the exterior representation formula (interior mesh)");
    if (m->has_pres)
      return fail(BEM_E_STATE, "the mesh has PRES elements, whose normal derivative is not c p: use bem_field_pv");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double* sc = scratch_on_current_device();
    int64_t* flag = reinterpret_cast<int64_t*>(sc);
    double* partial = sc + 1;
    const int64_t nb = (n_pts + kPointsPerBlock - 1) / kPointsPerBlock;
    if (n_pts > 0) {
      hipLaunchKernelGGL(k_flag_reset, dim3(1), dim3(64), 0, s, flag);
      // p_surf into tree order in the mesh's staging vector (allocated with the mesh)
      launch_gather(m->N, m->d_perm.p, reinterpret_cast<const double2*>(p_surf), m->d_x.p, s);
      launch_field(field_args(m, n_pts, 0), pts, m->d_x.p, reinterpret_cast<const double2*>(p_inc),
                   reinterpret_cast<double2*>(p_out), flag, s);
    }
    if (energy) {
      if (n_pts > 0)
        hipLaunchKernelGGL(k_energy_partials, dim3((unsigned)nb), dim3(kEnergyThreads), 0, s, n_pts,
                           kPointsPerBlock, reinterpret_cast<const double2*>(p_out), partial);
      hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kEnergyThreads), 0, s, (int)nb, partial, energy);
    }
    BEM_HIP(hipGetLastError());
    if (n_pts > 0) check_field_error(m, flag, s);
    return BEM_OK;
  });
}
