// Allocation-free batched solve: pdhcg_solve_batch with every device buffer
// of the batch (packed matrices and vectors, row partitions, parameter
// blocks, per-instance state, preconditioning factors) carved from one static
// device array instead of hipMalloc'd, for callers that cannot allocate
// device memory.  The solve itself is the batched kernel of the library.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.hpp"

namespace {

// Each GPU that runs this entry point holds its own copy of the array (the
// code object's device globals are per device) until the process ends.
__device__ __align__(256) char scratch[PDHCG_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_region[kMaxDevices];  // device address of `scratch` per device, looked up once

// The device address of the current device's `scratch`.  In host code the
// array's name is only a host-side stand-in, so every use below goes through
// the address that hipGetSymbolAddress returns with the device current.
int region_of_current_device(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return pdhcg::set_error(PDHCG_ERR_HIP, "pdhcg_solve_batch_noalloc: no current HIP device");
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_region[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return pdhcg::set_error(PDHCG_ERR_HIP, "pdhcg_solve_batch_noalloc: hipGetSymbolAddress of the static "
                                             "scratch failed");
    }
    g_region[dev] = (char*)p;
  }
  *out = g_region[dev];
  return 0;
}

}  // namespace

extern "C" int pdhcg_solve_batch_noalloc(int32_t count, const pdhcg_csr* Qs, const pdhcg_csr* As,
                                         const double* const* bs, const double* const* cs,
                                         const double* const* x0s, const double* const* y0s,
                                         double* const* x_outs, double* const* y_outs, pdhcg_result* rs,
                                         const pdhcg_settings* s, void* hip_stream) {
  if (count <= 0) return pdhcg::solve_batch_in_region(count, Qs, As, bs, cs, x0s, y0s, x_outs, y_outs, rs, s,
                                                       hip_stream, nullptr, 0);
  char* region = nullptr;
  const int rc = region_of_current_device(&region);
  if (rc) return rc;
  return pdhcg::solve_batch_in_region(count, Qs, As, bs, cs, x0s, y0s, x_outs, y_outs, rs, s, hip_stream, region,
                                      (size_t)PDHCG_NOALLOC_SCRATCH_BYTES);
}
