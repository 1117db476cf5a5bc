// The batched kernel: many independent QPs in one launch, one workgroup per QP
// (the same restarted PDHCG loop as the cooperative kernel, Alg. 1 with the
// rules of Sec. 4).  This translation unit compiles the shared device code for
// workgroups of kBatchBlock = 256 threads: two instances then share a CU, so
// the fixed latency of a small instance's iteration (a few dependent memory
// round trips per phase, tens of microseconds in all) is overlapped with
// another instance's work.
#define PDHCG_BATCH_UNIT 1
#include "solver.hpp"

namespace pdhcg {

// One workgroup per QP: workgroup g solves instance order[g] (the host sorts
// instances by decreasing work, so the dispatcher hands out the largest
// first).  Each workgroup runs the same loop as the cooperative kernel with
// nb = 1 (a grid barrier degenerates to a workgroup barrier), on its own slice
// of the packed matrices and vectors; dense Q blocks use the streaming dense
// product.  ||A|| comes from the same power iteration, per instance.
// Launched with kBlock threads but declared for 2 * kBlock: that bound holds
// the kernel and every function it calls to two waves per SIMD (256
// registers), the budget at which two workgroups fit on a CU; with the bound
// of the launch size alone the compiler takes the whole register file.
__global__ void __launch_bounds__(2 * kBlock) pdhcg_batch_kernel(BatchParams BP) {
  __shared__ double lds[kWaves * 16];
  __shared__ double svec[kDenseTile];
  const int idx = BP.order[blockIdx.x];
  __shared__ SolveParams Ps;
  // the partial sums of a phase go to LDS: with one workgroup per QP they
  // are read back only by the same workgroup, after a workgroup barrier
  __shared__ double part_lds[NSLOT];
  load_params(Ps, BP.params + idx, 0);
  if (threadIdx.x == 0) {  // this solve's partials, start point and warm-start fallback
    Ps.part = part_lds;
    const uint32_t gv = BP.given ? BP.given[idx] : 0u;
    if (!(gv & 1u)) Ps.x0 = nullptr;
    if (!(gv & 2u)) Ps.y0 = nullptr;
    if (!(gv & 3u) || !BP.warm_fallback) Ps.kkt_zero = 0.0;
  }
  __syncthreads();
  const SolveParams& P = Ps;
  Block B{0, 1, (int)threadIdx.x};
  GridSync gs{nullptr, 1u, 0};
  // start point (x0 or 0; y0 projected onto y >= 0, or 0)
  for (int j = B.tid; j < P.n; j += kBlock) {
    const double v = P.x0 ? P.x0[j] : 0.0;
    P.x[j] = v;
    P.xa[j] = v;
    P.x_anc[j] = v;
    if (BP.mixed) P.x32[j] = (float)v;
  }
  for (int i = B.tid; i < P.m; i += kBlock) {
    const double v = pos_part(P.y0 ? P.y0[i] : 0.0);
    P.y[i] = v;
    P.ya[i] = v;
    P.y_anc[i] = v;
  }
  __syncthreads();
  double nrm = 0.0;
  if (P.m > 0) power_norm(P.A, P.At, P.p0, P.p1, P.ax_avg, P.part, P.pt, P.pm, BP.power_iters, B, gs, lds, &nrm);
  __shared__ Ctl C;
  if (B.tid == 0) {
    SolverState& S = C.S;
    S = SolverState{};
    S.K_anchor = NAN;
    S.K_prev = INFINITY;
    S.omega = BP.pw_init;
    S.eta = BP.eta_factor / (nrm > 0.0 ? nrm : 1.0);
    S.tau = S.eta / S.omega;
    S.sigma = S.eta * S.omega;
    S.mixed = BP.mixed;
    S.t_start = *BP.t0;
    S.norm_A = nrm;
  }
  __syncthreads();
  if (P.Q.dense)
    drive<true>(P, B, gs, C, P.nb_inf, P.nc_inf, lds, svec, INT64_MAX);
  else
    drive<false>(P, B, gs, C, P.nb_inf, P.nc_inf, lds, svec, INT64_MAX);
  if (B.tid == 0) BP.st[idx] = C.S;
}

__global__ void batch_clock_kernel(uint64_t* t0) {
  if (threadIdx.x == 0) *t0 = wall_clock64();
}

hipError_t launch_batch(const BatchParams& p, int count, hipStream_t s) {
  hipLaunchKernelGGL(batch_clock_kernel, dim3(1), dim3(64), 0, s, p.t0);
  hipLaunchKernelGGL(pdhcg_batch_kernel, dim3(count), dim3(kBlock), 0, s, p);
  return hipGetLastError();
}

}  // namespace pdhcg
