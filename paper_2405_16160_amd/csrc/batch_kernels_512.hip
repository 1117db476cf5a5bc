// The batched kernel at 512 threads per workgroup (one instance per CU, LDS
// tiles of 4 096 entries and 1 024 rows): the alternative that the batch
// autotuner (pdhcg_batch_autotune) times against the 256-thread default of
// batch_kernels.hip; batches of large instances, which stream their data,
// can run faster with the wider workgroup.
#define PDHCG_BLOCK_SIZE 512
#include "solver.hpp"

namespace pdhcg {

__global__ void __launch_bounds__(kSolveBlock) pdhcg_batch_kernel_wg512(BatchParams BP) { batch_solve(BP); }

hipError_t launch_batch_512(const BatchParams& p, int count, hipStream_t s) {
  hipLaunchKernelGGL(pdhcg_batch_kernel_wg512, dim3(count), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

}  // namespace pdhcg
