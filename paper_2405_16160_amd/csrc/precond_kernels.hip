// Diagonal preconditioning of the data (Section 5, preprocessing).
//
// The factors belong to the symmetric matrix K = [[Q, A'], [A, 0]]: index
// i < n is variable i (row i of Q followed by row i of A'), index n + i is
// constraint i (row i of A).  A Ruiz step divides every row of K, and the
// column with the same index, by the square root of the row's largest
// magnitude; the Pock-Chambolle step (alpha = 1) divides by the square root
// of the row's 1-norm.  An all-zero row keeps factor 1.  After each step the
// factors are applied to Q, A and A' in place, each entry times f_i * f_j
// (the product is formed first, so Q stays exactly symmetric and A' stays
// the exact transpose of A).  The accumulated diagonal d holds D2 in d[0, n)
// and D1 in d[n, n + m).
//
// A one-time setup pass: one thread per row, rows in a grid-stride loop.
#include "device.hpp"

namespace pdhcg {

namespace {

__device__ __forceinline__ double row_stat(const int32_t* rp, const double* v, int64_t i, int mode, double acc) {
  const int32_t e = rp[i + 1];
  for (int32_t k = rp[i]; k < e; ++k) {
    const double a = fabs(v[k]);
    acc = mode == 0 ? fmax(acc, a) : acc + a;
  }
  return acc;
}

// f[i] = 1 / sqrt(stat of row i of K) (1 for a zero row), d[i] *= f[i];
// mode 0: largest magnitude, mode 1: 1-norm
__global__ void scale_factor_kernel(int64_t n, int64_t m, const int32_t* qrp, const double* qv, const int32_t* trp,
                                    const double* tv, const int32_t* arp, const double* av, int mode, double* f,
                                    double* d) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n + m; i += stride) {
    double s;
    if (i < n) {
      s = row_stat(qrp, qv, i, mode, 0.0);
      if (m > 0) s = row_stat(trp, tv, i, mode, s);
    } else {
      s = row_stat(arp, av, i - n, mode, 0.0);
    }
    const double fi = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
    f[i] = fi;
    d[i] *= fi;
  }
}

// val of row i, column j times fr[i] * fc[j]
__global__ void scale_apply_kernel(int64_t nrows, const int32_t* rp, const int32_t* col, double* val,
                                   const double* fr, const double* fc) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nrows; i += stride) {
    const double a = fr[i];
    const int32_t e = rp[i + 1];
    for (int32_t k = rp[i]; k < e; ++k) val[k] *= a * fc[col[k]];
  }
}

// out[i] = x[i] * s[i] (op 0) or x[i] / s[i] (op 1); out may be x
__global__ void diag_kernel(int64_t n, const double* x, const double* s, int op, double* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = op == 0 ? x[i] * s[i] : x[i] / s[i];
}

int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

hipError_t apply(const DevMat& M, const double* fr, const double* fc, hipStream_t s) {
  if (M.nrows == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_apply_kernel, dim3(grid_for(M.nrows)), dim3(kBlock), 0, s, (int64_t)M.nrows, M.rowptr,
                     M.col, const_cast<double*>(M.val), fr, fc);
  return hipGetLastError();
}

hipError_t step(const DevMat& Q, const DevMat& A, const DevMat& T, int mode, double* f, double* d, hipStream_t s) {
  const int64_t n = Q.nrows, m = A.nrows;
  hipLaunchKernelGGL(scale_factor_kernel, dim3(grid_for(n + m)), dim3(kBlock), 0, s, n, m, Q.rowptr, Q.val,
                     T.rowptr, T.val, A.rowptr, A.val, mode, f, d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = apply(Q, f, f, s)) != hipSuccess) return e;
  if ((e = apply(A, f + n, f, s)) != hipSuccess) return e;
  return apply(T, f, f + n, s);
}

}  // namespace

hipError_t launch_precondition(const DevMat& Q, const DevMat& A, const DevMat& T, int ruiz_iters, int pock_chambolle,
                               double* f, double* d, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (int it = 0; it < ruiz_iters && e == hipSuccess; ++it) e = step(Q, A, T, 0, f, d, s);
  if (e == hipSuccess && pock_chambolle) e = step(Q, A, T, 1, f, d, s);
  return e;
}

hipError_t launch_diag(const double* x, const double* scale, int64_t n, int op, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(diag_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, x, scale, op, out);
  return hipGetLastError();
}

}  // namespace pdhcg
