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
// the exact transpose of A).  The accumulated diagonals are D2 (n entries)
// and D1 (m entries).
//
// A one-time setup pass.  Each row is walked by a group of g lanes (a power
// of two up to 64, sized by the host to the mean row length) reading
// consecutive entries, so the loads of a group are coalesced and a long row
// costs len/g steps; the group combines its partial maxima or sums with lane
// exchanges.  Rows are taken in a grid-stride loop; all lanes of a group see
// the same row, so the exchanges only read active lanes.
#include "device.hpp"

namespace pdhcg {

namespace {

// this lane's share (entries lane, lane + g, ...) of row i's max or 1-norm
__device__ __forceinline__ double row_stat(const int32_t* rp, const double* v, int64_t i, int mode, int lane, int g,
                                           double acc) {
  const int32_t e = rp[i + 1];
  for (int32_t k = rp[i] + lane; k < e; k += g) {
    const double a = fabs(v[k]);
    acc = mode == 0 ? fmax(acc, a) : acc + a;
  }
  return acc;
}

// f[i] = 1 / sqrt(stat of row i of K) (1 for a zero row), and the factor is
// folded into D2[i] (i < n) or D1[i - n]; mode 0: largest magnitude, mode 1: 1-norm
__global__ void scale_factor_kernel(int64_t n, int64_t m, const int32_t* qrp, const double* qv, const int32_t* trp,
                                    const double* tv, const int32_t* arp, const double* av, int mode, int g,
                                    double* f, double* d2, double* d1) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = (int)(t & (g - 1));
  const int64_t stride = ((int64_t)gridDim.x * blockDim.x) / g;
  for (int64_t i = t / g; i < n + m; i += stride) {
    double s;
    if (i < n) {
      s = row_stat(qrp, qv, i, mode, lane, g, 0.0);
      if (m > 0) s = row_stat(trp, tv, i, mode, lane, g, s);
    } else {
      s = row_stat(arp, av, i - n, mode, lane, g, 0.0);
    }
    for (int off = g >> 1; off > 0; off >>= 1) {
      const double o = __shfl_xor(s, off, g);
      s = mode == 0 ? fmax(s, o) : s + o;
    }
    if (lane == 0) {
      const double fi = s > 0.0 ? 1.0 / sqrt(s) : 1.0;
      f[i] = fi;
      if (i < n)
        d2[i] *= fi;
      else
        d1[i - n] *= fi;
    }
  }
}

// val of row i, column j times fr[i] * fc[j]
__global__ void scale_apply_kernel(int64_t nrows, const int32_t* rp, const int32_t* col, double* val,
                                   const double* fr, const double* fc, int g) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int lane = (int)(t & (g - 1));
  const int64_t stride = ((int64_t)gridDim.x * blockDim.x) / g;
  for (int64_t i = t / g; i < nrows; i += stride) {
    const double a = fr[i];
    const int32_t e = rp[i + 1];
    for (int32_t k = rp[i] + lane; k < e; k += g) val[k] *= a * fc[col[k]];
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

// lanes per row: the power of two nearest above the mean row length, 1..64
int lanes_for(int64_t nnz, int64_t nrows) {
  const double mean = nrows > 0 ? (double)nnz / (double)nrows : 1.0;
  int g = 1;
  while (g < 64 && g < mean) g <<= 1;
  return g;
}

struct Groups {
  int q, a, t, k;  // lanes per row of Q, A, A' and of the rows of K
};

hipError_t apply(const DevMat& M, int64_t nnz, const double* fr, const double* fc, int g, hipStream_t s) {
  if (M.nrows == 0 || nnz == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_apply_kernel, dim3(grid_for((int64_t)M.nrows * g)), dim3(kBlock), 0, s, (int64_t)M.nrows,
                     M.rowptr, M.col, const_cast<double*>(M.val), fr, fc, g);
  return hipGetLastError();
}

hipError_t step(const DevMat& Q, const DevMat& A, const DevMat& T, int64_t nnzq, int64_t nnza, const Groups& G,
                int mode, double* f, double* d2, double* d1, hipStream_t s) {
  const int64_t n = Q.nrows, m = A.nrows;
  hipLaunchKernelGGL(scale_factor_kernel, dim3(grid_for((n + m) * G.k)), dim3(kBlock), 0, s, n, m, Q.rowptr, Q.val,
                     T.rowptr, T.val, A.rowptr, A.val, mode, G.k, f, d2, d1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = apply(Q, nnzq, f, f, G.q, s)) != hipSuccess) return e;
  if ((e = apply(A, nnza, f + n, f, G.a, s)) != hipSuccess) return e;
  return apply(T, nnza, f, f + n, G.t, s);
}

}  // namespace

hipError_t launch_precondition(const DevMat& Q, const DevMat& A, const DevMat& T, int64_t nnzq, int64_t nnza,
                               int ruiz_iters, int pock_chambolle, double* f, double* d2, double* d1, hipStream_t s) {
  Groups G;
  G.q = lanes_for(nnzq, Q.nrows);
  G.a = lanes_for(nnza, A.nrows);
  G.t = lanes_for(nnza, T.nrows);
  G.k = lanes_for(nnzq + 2 * nnza, (int64_t)Q.nrows + A.nrows);
  hipError_t e = hipSuccess;
  for (int it = 0; it < ruiz_iters && e == hipSuccess; ++it) e = step(Q, A, T, nnzq, nnza, G, 0, f, d2, d1, s);
  if (e == hipSuccess && pock_chambolle) e = step(Q, A, T, nnzq, nnza, G, 1, f, d2, d1, s);
  return e;
}

hipError_t launch_diag(const double* x, const double* scale, int64_t n, int op, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(diag_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, n, x, scale, op, out);
  return hipGetLastError();
}

}  // namespace pdhcg
