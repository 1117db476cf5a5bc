// Diagonal preconditioning of the data (Sec. 4, preprocessing).
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

// ------------------------------------------------------------ batched form
//
// One workgroup per instance of a batch runs all steps on that instance's
// blocks, with workgroup barriers between the passes of a step: the factor
// statistics of every index of K, the factors (folded into D2, D1), then the
// scaling of Q, A and A' in place.  Q is a CSR block, a dense n x n block, or
// a factor [F (n x k) | F' (k x n) | d (n)] of Q = F F' + diag(d); for the
// factor the row statistics of F F' + diag(d) are formed from F in tiles
// (the entries of Q are never stored), and the scaling keeps the form:
// diag(f) (F F' + diag(d)) diag(f) = (diag(f) F)(diag(f) F)' + diag(f^2 d).

__device__ __forceinline__ double stat_comb(double a, double b, int mode) { return mode == 0 ? fmax(a, b) : a + b; }

// statistic of every row of F F' + diag(d), combined into st[0 .. n): tiles
// of 128 rows x 64 columns, F staged in LDS in chunks of 32 of its columns,
// 4 x 4 products per thread; the 16 lanes that share rows combine their
// partial statistics with lane exchanges
constexpr int kFtJ = 128, kFtK = 64, kFtL = 32;

__device__ void factor_row_stats(const double* F, const double* d, int n, int k, int mode, double* st,
                                 double* lds) {
  double* Fj = lds;               // [kFtL][kFtJ]
  double* Fk = lds + kFtL * kFtJ;  // [kFtL][kFtK]
  const int tid = (int)threadIdx.x;
  const int tj = tid / 16, tk = tid % 16;  // rows tj*4 .. +3, columns tk*4 .. +3 of a tile
  for (int j0 = 0; j0 < n; j0 += kFtJ) {
    double rs[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < n; k0 += kFtK) {
      double acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
      for (int l0 = 0; l0 < k; l0 += kFtL) {
        __syncthreads();
        for (int e = tid; e < kFtJ * kFtL; e += kBlock) {
          const int row = e / kFtL, l = e % kFtL, gr = j0 + row, gl = l0 + l;
          Fj[l * kFtJ + row] = (gr < n && gl < k) ? F[(int64_t)gr * k + gl] : 0.0;
        }
        for (int e = tid; e < kFtK * kFtL; e += kBlock) {
          const int row = e / kFtL, l = e % kFtL, gr = k0 + row, gl = l0 + l;
          Fk[l * kFtK + row] = (gr < n && gl < k) ? F[(int64_t)gr * k + gl] : 0.0;
        }
        __syncthreads();
        for (int l = 0; l < kFtL; ++l) {
          const double2* pa = (const double2*)(Fj + l * kFtJ + tj * 4);
          const double2* pb = (const double2*)(Fk + l * kFtK + tk * 4);
          const double2 a01 = pa[0], a23 = pa[1], b01 = pb[0], b23 = pb[1];
          const double a[4] = {a01.x, a01.y, a23.x, a23.y}, b[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int gr = j0 + tj * 4 + r, gc = k0 + tk * 4 + c;
          if (gr < n && gc < n) rs[r] = stat_comb(rs[r], fabs(acc[r][c] + (gr == gc ? d[gr] : 0.0)), mode);
        }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
      for (int off = 8; off > 0; off >>= 1) rs[r] = stat_comb(rs[r], __shfl_xor(rs[r], off, 16), mode);
    if (tk == 0)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = j0 + tj * 4 + r;
        if (gr < n) st[gr] = stat_comb(st[gr], rs[r], mode);
      }
  }
}

__global__ void __launch_bounds__(kBlock) batch_precondition_kernel(const PrecInst* insts, int ruiz_iters,
                                                                    int pock_chambolle) {
  __shared__ __align__(16) double lds[kFtL * (kFtJ + kFtK)];
  const PrecInst I = insts[blockIdx.x];
  const int n = I.n, m = I.m, tid = (int)threadIdx.x;
  double* const f = I.f;  // statistics, then factors: n entries of the variables, then m of the rows
  for (int step = 0; step < ruiz_iters + pock_chambolle; ++step) {
    const int mode = step < ruiz_iters ? 0 : 1;
    // CSR rows of K: Q (when CSR) and A' for a variable, A for a row
    {
      const int g = I.gk, lane = tid & (g - 1);
      for (int i = tid / g; i < n + m; i += kBlock / g) {
        double sv;
        if (i < n) {
          sv = I.qkind == 0 ? row_stat(I.qrp, I.qval, i, mode, lane, g, 0.0) : 0.0;
          if (m > 0) sv = row_stat(I.trp, I.tval, i, mode, lane, g, sv);
        } else {
          sv = row_stat(I.arp, I.aval, i - n, mode, lane, g, 0.0);
        }
        for (int off = g >> 1; off > 0; off >>= 1) sv = stat_comb(sv, __shfl_xor(sv, off, g), mode);
        if (lane == 0) f[i] = sv;
      }
    }
    __syncthreads();
    if (I.qkind == 1) {  // dense symmetric Q: the statistic of row c is that of column c
      for (int c = tid; c < n; c += kBlock) {
        double sv = 0.0;
        for (int r = 0; r < n; ++r) sv = stat_comb(sv, fabs(I.qval[(int64_t)r * n + c]), mode);
        f[c] = stat_comb(f[c], sv, mode);
      }
    } else if (I.qkind == 2) {
      factor_row_stats(I.qval, I.qval + 2 * (int64_t)n * I.k, n, I.k, mode, f, lds);
    }
    __syncthreads();
    for (int i = tid; i < n + m; i += kBlock) {
      const double sv = f[i];
      const double fi = sv > 0.0 ? 1.0 / sqrt(sv) : 1.0;
      f[i] = fi;
      if (i < n)
        I.d2[i] *= fi;
      else
        I.d1[i - n] *= fi;
    }
    __syncthreads();
    // scale in place: entry (i, j) times f_i * f_j
    if (I.qkind == 0) {
      const int g = I.gq, lane = tid & (g - 1);
      for (int i = tid / g; i < n; i += kBlock / g) {
        const double a = f[i];
        for (int32_t e = I.qrp[i] + lane; e < I.qrp[i + 1]; e += g) I.qval[e] *= a * f[I.qcol[e]];
      }
    } else if (I.qkind == 1) {
      for (int r = 0; r < n; ++r) {
        const double a = f[r];
        for (int c = tid; c < n; c += kBlock) I.qval[(int64_t)r * n + c] *= a * f[c];
      }
    } else {
      const int k = I.k;
      double* F = I.qval;
      double* Ft = F + (int64_t)n * k;
      double* dd = Ft + (int64_t)k * n;
      for (int64_t e = tid; e < (int64_t)n * k; e += kBlock) {
        F[e] *= f[e / k];
        Ft[e] *= f[e % n];
      }
      for (int j = tid; j < n; j += kBlock) dd[j] *= f[j] * f[j];
    }
    if (m > 0) {
      const int ga = I.ga, la = tid & (ga - 1);
      for (int i = tid / ga; i < m; i += kBlock / ga) {
        const double a = f[n + i];
        for (int32_t e = I.arp[i] + la; e < I.arp[i + 1]; e += ga) I.aval[e] *= a * f[I.acol[e]];
      }
      const int gt = I.gt, lt = tid & (gt - 1);
      for (int j = tid / gt; j < n; j += kBlock / gt) {
        const double a = f[j];
        for (int32_t e = I.trp[j] + lt; e < I.trp[j + 1]; e += gt) I.tval[e] *= a * f[n + I.tcol[e]];
      }
    }
    __syncthreads();
  }
}

}  // namespace

int precond_lanes(int64_t nnz, int64_t nrows) { return lanes_for(nnz, nrows); }

hipError_t launch_batch_precondition(const PrecInst* insts, int count, int ruiz_iters, int pock_chambolle,
                                     hipStream_t s) {
  if (count <= 0 || ruiz_iters + pock_chambolle <= 0) return hipSuccess;
  hipLaunchKernelGGL(batch_precondition_kernel, dim3(count), dim3(kBlock), 0, s, insts, ruiz_iters, pock_chambolle);
  return hipGetLastError();
}

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
