// Persistent cooperative kernel for one QP: the whole restarted PDHCG loop
// (Alg. 1 with the practical rules of Sec. 4) runs on the device.  Each
// workgroup owns fixed row ranges of Q, A' and A; phases are separated by
// grid barriers; scalars (CG alpha/beta/rho, relKKT, restart tests, step
// sizes) are FP64 and computed redundantly by every workgroup from the same
// per-workgroup partials, so every workgroup takes the same branch.
#include "solver.hpp"

namespace pdhcg {
namespace {

// Copy the workgroup's rows of M (row pointers, columns, values of vbytes)
// into its resident block at base and record the block in w.
__device__ void place_resident(WgPart& w, const DevMat& M, char* base, int vbytes) {
  const int nr = w.r1 - w.r0;
  const int e0 = M.rowptr[w.r0], ne = M.rowptr[w.r1] - e0;
  int32_t* lrp = (int32_t*)base;
  int32_t* lcol = (int32_t*)(base + align16(4 * (int64_t)(nr + 1)));
  char* lval = (char*)lcol + align16(4 * (int64_t)ne);
  for (int j = threadIdx.x; j <= nr; j += kBlock) lrp[j] = gld(M.rowptr + w.r0 + j);
  for (int k = threadIdx.x; k < ne; k += kBlock) lcol[k] = gld(M.col + e0 + k);
  if (vbytes == 4)
    for (int k = threadIdx.x; k < ne; k += kBlock) ((float*)lval)[k] = gld(M.val32 + e0 + k);
  else
    for (int k = threadIdx.x; k < ne; k += kBlock) ((double*)lval)[k] = gld(M.val + e0 + k);
  if (threadIdx.x == 0) {
    w.e0 = e0;
    w.lrp = lrp;
    w.lcol = lcol;
    w.lval = lval;
  }
}

}  // namespace

__global__ void __launch_bounds__(kBlock) pdhcg_solve_kernel(const SolveParams* __restrict__ Pg) {
  __shared__ SolveParams Ps;
  extern __shared__ __align__(16) char dyn_lds[];
  load_params(Ps, Pg, (int)blockIdx.x);
  if (Ps.res_cg) place_resident(Ps.w_cg, Ps.Q, dyn_lds, Ps.res_vbytes);
  if (Ps.res_m) place_resident(Ps.w_m, Ps.A, dyn_lds + Ps.res_m_off, Ps.res_vbytes);
  if (threadIdx.x == 0) Ps.cg_own = Ps.own_cg ? (double*)(dyn_lds + Ps.own_off) : nullptr;
  __syncthreads();
  const SolveParams& P = Ps;
  const double nb_inf = P.nb_inf, nc_inf = P.nc_inf;
  __shared__ double lds[kWaves * 16];
  Block B{(int)blockIdx.x, (int)gridDim.x, (int)threadIdx.x};
  GridSync gs{P.bar, (uint32_t)gridDim.x, 0};
  if (!gs.init()) {
    if (B.b == 0 && B.tid == 0) P.st->done = -1;  // barrier failure: reported as a HIP error
    return;
  }
  __shared__ Ctl C;
  if (B.tid == 0) C.S = *P.st;
  __syncthreads();
  if (C.S.done) return;
  const bool ok = drive<false>(P, B, gs, C, nb_inf, nc_inf, lds, nullptr, P.iters_this_launch);
  if (B.b == 0 && B.tid == 0) {
    if (!ok)
      P.st->done = -1;  // barrier failure: reported as a HIP error
    else
      *P.st = C.S;
  }
}

// -------------------------------------------------------- power iteration

__global__ void __launch_bounds__(kBlock) pdhcg_power_kernel(PowerParams P) {
  __shared__ double lds[kWaves * 8];
  Block B{(int)blockIdx.x, (int)gridDim.x, (int)threadIdx.x};
  GridSync gs{P.bar, (uint32_t)gridDim.x, 0};
  if (!gs.init()) return;  // (the host finds the abort word raised)
  double nrm = 0.0;
  if (power_norm(P.A, P.At, P.v, P.w, P.u, P.part, P.pn, P.pm, P.iters, B, gs, lds, &nrm) && B.b == 0 &&
      B.tid == 0)
    P.out[0] = nrm;
}

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

hipError_t launch_solve(const SolveParams* p_dev, int nb, int dyn_lds, hipStream_t s) {
  const SolveParams* pc = p_dev;
  void* args[] = {&pc};
  if (dyn_lds > 0) {
    hipError_t e = hipFuncSetAttribute((const void*)pdhcg_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       dyn_lds);
    if (e != hipSuccess) return e;
  }
  return hipLaunchCooperativeKernel((const void*)pdhcg_solve_kernel, dim3(nb), dim3(kBlock), args,
                                    (unsigned)dyn_lds, s);
}

hipError_t solve_kernel_lds(int* static_bytes) {
  hipFuncAttributes a;
  hipError_t e = hipFuncGetAttributes(&a, (const void*)pdhcg_solve_kernel);
  if (e != hipSuccess) return e;
  *static_bytes = (int)a.sharedSizeBytes;
  return hipSuccess;
}

hipError_t solve_occupancy_dyn(int dyn_lds, int* per_cu) {
  if (dyn_lds > 0) {
    hipError_t e = hipFuncSetAttribute((const void*)pdhcg_solve_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       dyn_lds);
    if (e != hipSuccess) return e;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, (const void*)pdhcg_solve_kernel, kBlock, dyn_lds);
}

hipError_t launch_power(const PowerParams& p, int nb, hipStream_t s) {
  PowerParams pc = p;
  void* args[] = {&pc};
  return hipLaunchCooperativeKernel((const void*)pdhcg_power_kernel, dim3(nb), dim3(kBlock), args, 0, s);
}

hipError_t launch_init_point(const SolveParams* p_dev, int64_t n, int64_t m, hipStream_t s) {
  int64_t len = n > m ? n : m;
  int grid = (int)((len + kBlock - 1) / kBlock);
  if (grid < 1) grid = 1;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(init_point_kernel, dim3(grid), dim3(kBlock), 0, s, p_dev);
  return hipGetLastError();
}

hipError_t solve_occupancy(int* per_cu) {
  int a = 0, b = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, (const void*)pdhcg_solve_kernel, kBlock, 0);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void*)pdhcg_power_kernel, kBlock, 0);
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
