// The cooperative solve kernel and the power iteration compiled for 256-thread
// workgroups, two per CU (the device code of solver.hpp at that size, LDS
// tiles of 2 048 entries).
// The planner takes it for QPs whose gathered vectors stream from the
// last-level cache (the textbook CG form's sizes): a CU holds eight waves
// either way, but two workgroups wait apart, so one's gathers stay in flight
// while the other sums a tile or waits at a workgroup barrier, at the cost of
// twice the arrivals at every grid barrier.
#define PDHCG_BLOCK_SIZE 256
#include "solver.hpp"

namespace pdhcg {

// Launched with kBlock threads but declared for kSolveBlock: two waves per
// SIMD (256 registers) for the kernel and every function it calls, the
// budget at which two workgroups fit on a CU.
__global__ void __launch_bounds__(kSolveBlock) pdhcg_solve_kernel_wg256(const SolveParams* __restrict__ Pg) {
  solve_body(Pg);
}

__global__ void __launch_bounds__(kSolveBlock) pdhcg_power_kernel_wg256(PowerParams P) { power_body(P); }

const void* solve_kernel_256() { return (const void*)pdhcg_solve_kernel_wg256; }
const void* power_kernel_256() { return (const void*)pdhcg_power_kernel_wg256; }

}  // namespace pdhcg
