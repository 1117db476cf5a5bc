// Persistent cooperative kernel for one QP: the whole restarted PDHCG loop
// (Alg. 1 with the practical rules of Sec. 4) runs on the device.  Each
// workgroup owns fixed row ranges of Q, A' and A; phases are separated by
// grid barriers; scalars (CG alpha/beta/rho, relKKT, restart tests, step
// sizes) are FP64 and computed redundantly by every workgroup from the same
// per-workgroup partials, so every workgroup takes the same branch.
#include "solver.hpp"

namespace pdhcg {

__global__ void __launch_bounds__(kBlock) pdhcg_solve_kernel(const SolveParams* __restrict__ Pg) { solve_body(Pg); }

// -------------------------------------------------------- power iteration

__global__ void __launch_bounds__(kBlock) pdhcg_power_kernel(PowerParams P) { power_body(P); }

// ------------------------------------------------------ small helper kernels

__global__ void init_point_kernel(const SolveParams* __restrict__ Pg) {
  const SolveParams& P = *Pg;
  const double* x0 = P.x0;
  const double* y0 = P.y0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < P.n; j += stride) {
    const double v = x0 ? x0[j] : 0.0;
    P.x[j] = v;
    P.xa[j] = v;
    P.x_anc[j] = v;
    if (P.x32) P.x32[j] = (float)v;
  }
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P.m; i += stride) {
    double v = y0 ? y0[i] : 0.0;
    v = v > 0.0 ? v : (v == v ? 0.0 : v);
    P.y[i] = v;
    P.ya[i] = v;
    P.y_anc[i] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) P.st->t_start = wall_clock64();
}

__global__ void to_f32_kernel(const double* in, float* out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += stride) out[j] = (float)in[j];
}

// ---------------------------------------------------------------- launchers

// the solve kernel for `threads` per workgroup: this unit's (512 threads), or
// the 256-thread copy of solve_kernels_256.hip
static const void* solve_kernel_for(int threads) {
  return threads == kBlock ? (const void*)pdhcg_solve_kernel : solve_kernel_256();
}

// the power iteration at the same workgroup size (it walks the same row
// partitions, whose tiles are sized for it)
static const void* power_kernel_for(int threads) {
  return threads == kBlock ? (const void*)pdhcg_power_kernel : power_kernel_256();
}

hipError_t launch_solve(int threads, const SolveParams* p_dev, int nb, int dyn_lds, hipStream_t s) {
  const SolveParams* pc = p_dev;
  void* args[] = {&pc};
  const void* k = solve_kernel_for(threads);
  if (dyn_lds > 0) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_lds);
    if (e != hipSuccess) return e;
  }
  return hipLaunchCooperativeKernel(k, dim3(nb), dim3(threads), args, (unsigned)dyn_lds, s);
}

hipError_t solve_kernel_lds(int threads, int* static_bytes) {
  hipFuncAttributes a;
  hipError_t e = hipFuncGetAttributes(&a, solve_kernel_for(threads));
  if (e != hipSuccess) return e;
  *static_bytes = (int)a.sharedSizeBytes;
  return hipSuccess;
}

hipError_t solve_occupancy_dyn(int threads, int dyn_lds, int* per_cu) {
  const void* k = solve_kernel_for(threads);
  if (dyn_lds > 0) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, dyn_lds);
    if (e != hipSuccess) return e;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k, threads, dyn_lds);
}

hipError_t launch_power(int threads, const PowerParams& p, int nb, hipStream_t s) {
  PowerParams pc = p;
  void* args[] = {&pc};
  return hipLaunchCooperativeKernel(power_kernel_for(threads), dim3(nb), dim3(threads), args, 0, s);
}

hipError_t launch_init_point(const SolveParams* p_dev, int64_t n, int64_t m, hipStream_t s) {
  int64_t len = n > m ? n : m;
  int grid = (int)((len + kBlock - 1) / kBlock);
  if (grid < 1) grid = 1;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(init_point_kernel, dim3(grid), dim3(kBlock), 0, s, p_dev);
  return hipGetLastError();
}

hipError_t solve_occupancy(int threads, int* per_cu) {
  int a = 0, b = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, solve_kernel_for(threads), threads, 0);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, power_kernel_for(threads), threads, 0);
  if (e != hipSuccess) return e;
  *per_cu = a < b ? a : b;
  return hipSuccess;
}

hipError_t launch_to_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  int grid = (int)((n + kBlock - 1) / kBlock);
  if (grid < 1) grid = 1;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(to_f32_kernel, dim3(grid), dim3(kBlock), 0, s, in, out, n);
  return hipGetLastError();
}
}  // namespace pdhcg
