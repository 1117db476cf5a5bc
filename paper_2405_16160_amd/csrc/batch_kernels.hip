// The batched kernel: many independent QPs in one launch, one workgroup per QP
// (the same restarted PDHCG loop as the cooperative kernel, Alg. 1 with the
// rules of Sec. 4; the loop itself is batch_solve in solver.hpp).  This
// translation unit compiles the shared device code for workgroups of 256
// threads, the default: two instances then share a CU, so the fixed latency
// of a small instance's iteration (a few dependent memory round trips per
// phase, tens of microseconds in all) is overlapped with another instance's
// work.  batch_kernels_512.hip holds the same kernel at 512 threads.
#define PDHCG_BLOCK_SIZE 256
#include "solver.hpp"

namespace pdhcg {

// Launched with kBlock threads but declared for 512: that bound holds the
// kernel and every function it calls to two waves per SIMD (256 registers),
// the budget at which two workgroups fit on a CU; with the bound of the
// launch size alone the compiler takes the whole register file.
__global__ void __launch_bounds__(kSolveBlock) pdhcg_batch_kernel(BatchParams BP) { batch_solve(BP); }

__global__ void batch_clock_kernel(uint64_t* t0) {
  if (threadIdx.x == 0) *t0 = wall_clock64();
}

hipError_t launch_batch_clock(uint64_t* t0, hipStream_t s) {
  hipLaunchKernelGGL(batch_clock_kernel, dim3(1), dim3(64), 0, s, t0);
  return hipGetLastError();
}

hipError_t launch_batch_256(const BatchParams& p, int count, hipStream_t s) {
  hipLaunchKernelGGL(pdhcg_batch_kernel, dim3(count), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

}  // namespace pdhcg
