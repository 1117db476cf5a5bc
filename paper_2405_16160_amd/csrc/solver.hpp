// Device code of the restarted PDHCG loop shared by the cooperative single-QP
// kernel (solve_kernels.hip) and the batched kernel (batch_kernels.hip): the
// phases, the control state machine, the driver and the power iteration.
// Every workgroup-size-dependent constant comes from internal.hpp, so each
// including translation unit compiles its own copy for its workgroup size;
// everything here has internal linkage for that reason.
#pragma once
#include <math.h>

#include "device.hpp"

namespace pdhcg {

namespace {

struct Block {
  int b, nb, tid;
};

__device__ __forceinline__ double rel_div(double num, double den) { return num / (1.0 + den); }

// (v)^+ that keeps a NaN visible
__device__ __forceinline__ double pos_part(double v) { return v > 0.0 ? v : (v == v ? 0.0 : v); }

// ------------------------------------------------------------------ phases

// One workgroup computes out_i = sum_j M[i,j] v_j for a dense symmetric n x n
// matrix stored row-major.  Symmetry lets thread t own rows i = t + kBlock*k
// and stream M row by row: for each j the workgroup reads M[j, i0..] (=
// M[i0.., j]) with unit stride across threads, and v_j is broadcast from an
// LDS tile.  No cross-lane reduction is needed.  gen(j) produces v_j (FP64)
// and is called once per j per row pass; epi(i, sum) receives each row.
// One pass of a dense product over rows i0 + tid + k * kBlock, k < K (rows
// clamped into range: surplus rows are computed and dropped, so every load
// is unconditional and kJ * K of them are in flight per thread).
// The pass is written for a rectangular M (nr rows streamed, nc columns
// owned, row-major): out_c = sum_j M[j, c] v_j, which for a symmetric square M
// is the product M v and for a tall factor F gives F' v.
template <int K, typename V, typename Gen>
__device__ __forceinline__ void dense_pass(const V* M, int nr, int nc, int i0, double* svec, Gen& gen,
                                           double* acc) {
  constexpr int kJ = 8;  // rows per unrolled step
  int ic[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    acc[k] = 0.0;
    ic[k] = min(i0 + (int)threadIdx.x + k * kBlock, nc - 1);
  }
  for (int j0 = 0; j0 < nr; j0 += kDenseTile) {
    const int jt = nr - j0 < kDenseTile ? nr - j0 : kDenseTile;
    __syncthreads();
    for (int j = threadIdx.x; j < jt; j += kBlock) svec[j] = gen(j0 + j, i0 == 0);
    __syncthreads();
    const V* base = M + (int64_t)j0 * nc;
    int j = 0;
    for (; j + kJ <= jt; j += kJ) {
      V v[kJ][K];
#pragma unroll
      for (int jj = 0; jj < kJ; ++jj)
#pragma unroll
        for (int k = 0; k < K; ++k) v[jj][k] = gld(base + (int64_t)(j + jj) * nc + ic[k]);
#pragma unroll
      for (int jj = 0; jj < kJ; ++jj) {
        const double sj = svec[j + jj];
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += (double)v[jj][k] * sj;
      }
    }
    for (; j < jt; ++j) {
      const double sj = svec[j];
#pragma unroll
      for (int k = 0; k < K; ++k) acc[k] += (double)gld(base + (int64_t)j * nc + ic[k]) * sj;
    }
  }
}

// The FP32 form of dense_pass with 16-byte loads: thread t owns the four
// consecutive columns i0 + 4t .. i0 + 4t + 3 (a pass covers 4 kBlock
// columns), kJ rows in flight per step (16 loads of 16 bytes, where the
// FP64-value form has 8 x K loads of 8 bytes).  Each column still adds the
// rows in order, so the sums are those of dense_pass.  A thread whose four
// columns run past nc reads up to three values beyond its row: the next row,
// or what follows the matrix in its block (F' after F, d after F'), or the
// padding of the packed FP32 value array after the last matrix; those columns
// are dropped.  A thread with no column below nc reads its row's start.
template <typename Gen>
__device__ __forceinline__ void dense_pass4(const float* M, int nr, int nc, int i0, double* svec, Gen& gen,
                                            double* acc) {
  constexpr int kJ = 16;  // rows per unrolled step
  const int c0 = i0 + 4 * (int)threadIdx.x;
  const int cl = c0 < nc ? c0 : 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = 0.0;
  for (int j0 = 0; j0 < nr; j0 += kDenseTile) {
    const int jt = nr - j0 < kDenseTile ? nr - j0 : kDenseTile;
    __syncthreads();
    for (int j = threadIdx.x; j < jt; j += kBlock) svec[j] = gen(j0 + j, i0 == 0);
    __syncthreads();
    const float* base = M + (int64_t)j0 * nc + cl;
    int j = 0;
    for (; j + kJ <= jt; j += kJ) {
      f32x4u v[kJ];
#pragma unroll
      for (int jj = 0; jj < kJ; ++jj) v[jj] = gld4(base + (int64_t)(j + jj) * nc);
#pragma unroll
      for (int jj = 0; jj < kJ; ++jj) {
        const double sj = svec[j + jj];
        acc[0] += (double)v[jj].x * sj;
        acc[1] += (double)v[jj].y * sj;
        acc[2] += (double)v[jj].z * sj;
        acc[3] += (double)v[jj].w * sj;
      }
    }
    for (; j < jt; ++j) {
      const double sj = svec[j];
      const f32x4u v = gld4(base + (int64_t)j * nc);
      acc[0] += (double)v.x * sj;
      acc[1] += (double)v.y * sj;
      acc[2] += (double)v.z * sj;
      acc[3] += (double)v.w * sj;
    }
  }
}

// out_c = sum_j M[j, c] v_j for all c < nc, v_j = gen(j, first) (first: the
// first column pass, where gen may store what it forms), epi(c, out_c)
template <typename V, typename Gen, typename Epi>
__device__ void rect_rows(const V* M, int nr, int nc, double* svec, Gen& gen, Epi& epi) {
  if constexpr (sizeof(V) == 4) {
    for (int i0 = 0; i0 < nc; i0 += 4 * kBlock) {
      double acc[4];
      dense_pass4(M, nr, nc, i0, svec, gen, acc);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + 4 * (int)threadIdx.x + q;
        if (i < nc) epi(i, acc[q]);
      }
    }
    __syncthreads();
    return;
  }
  for (int i0 = 0; i0 < nc; i0 += kBlock * kDenseRows) {
    double acc[kDenseRows];
    const int cols = nc - i0;
    const int K = cols > 3 * kBlock ? 4 : (cols > 2 * kBlock ? 3 : (cols > kBlock ? 2 : 1));  // uniform
    if (K == 4) dense_pass<4>(M, nr, nc, i0, svec, gen, acc);
    else if (K == 3) dense_pass<3>(M, nr, nc, i0, svec, gen, acc);
    else if (K == 2) dense_pass<2>(M, nr, nc, i0, svec, gen, acc);
    else dense_pass<1>(M, nr, nc, i0, svec, gen, acc);
#pragma unroll
    for (int k = 0; k < kDenseRows; ++k) {
      const int i = i0 + (int)threadIdx.x + k * kBlock;
      if (k < K && i < nc) epi(i, acc[k]);
    }
  }
  __syncthreads();
}

// t = F' v for a factor with k <= 256 columns and n <= kDenseTile rows, v
// already in svec (F read with the non-temporal hint: on the benchmark batch
// that keeps the A-side data and vectors cached, 1.7 % less kernel time;
// on the F' pass of the second product it costs time): wave w takes rows w, w + kWaves, ... and its lanes the
// columns lane + 64 q (all waves busy, where one thread per column would
// leave most of them idle); the waves' partial sums are added in LDS in a
// fixed order.  red holds kWaves * 256 doubles.
template <int Q4, typename V>
__device__ void factor_tv(const V* F, int n, int k, const double* svec, double* red, double* t) {
  constexpr int kJ = 8;  // rows per unrolled step (per wave)
  const int tid = (int)threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  double acc[Q4];
  int cc[Q4];
#pragma unroll
  for (int q = 0; q < Q4; ++q) {
    acc[q] = 0.0;
    cc[q] = min(lane + kWave * q, k - 1);
  }
  for (int j = w; j < n; j += kWaves * kJ) {
    V u[kJ][Q4];
#pragma unroll
    for (int jj = 0; jj < kJ; ++jj) {
      const int row = min(j + kWaves * jj, n - 1);
#pragma unroll
      for (int q = 0; q < Q4; ++q) u[jj][q] = gld_nt(F + (int64_t)row * k + cc[q]);
    }
#pragma unroll
    for (int jj = 0; jj < kJ; ++jj) {
      const int row = j + kWaves * jj;
      const double vj = row < n ? svec[row] : 0.0;
#pragma unroll
      for (int q = 0; q < Q4; ++q) acc[q] += (double)u[jj][q] * vj;
    }
  }
#pragma unroll
  for (int q = 0; q < Q4; ++q) {
    const int c = lane + kWave * q;
    if (c < k) red[w * 256 + c] = acc[q];
  }
  __syncthreads();
  for (int c = tid; c < k; c += kBlock) {
    double sum = red[c];
    for (int ww = 1; ww < kWaves; ++ww) sum += red[ww * 256 + c];
    t[c] = sum;
  }
  __syncthreads();
}

// factor_tv for FP32 factors with 16-byte loads: lane l takes the columns
// 4l .. 4l + 3 of every row of its wave (k <= 256), 16 rows in flight per
// step; each column adds its rows in the same order as factor_tv, so t is the
// same.  A lane whose columns run past k reads up to three values beyond the
// row (the next row, or F' after the last row); those are dropped.
__device__ void factor_tv4(const float* F, int n, int k, const double* svec, double* red, double* t) {
  constexpr int kJ = 16;  // rows per unrolled step (per wave)
  const int tid = (int)threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int c0 = 4 * lane;
  const int cl = c0 < k ? c0 : 0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = w; j < n; j += kWaves * kJ) {
    f32x4u u[kJ];
#pragma unroll
    for (int jj = 0; jj < kJ; ++jj) {
      const int row = min(j + kWaves * jj, n - 1);
      u[jj] = gld4_nt(F + (int64_t)row * k + cl);
    }
#pragma unroll
    for (int jj = 0; jj < kJ; ++jj) {
      const int row = j + kWaves * jj;
      const double vj = row < n ? svec[row] : 0.0;
      acc[0] += (double)u[jj].x * vj;
      acc[1] += (double)u[jj].y * vj;
      acc[2] += (double)u[jj].z * vj;
      acc[3] += (double)u[jj].w * vj;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = c0 + q;
    if (c < k) red[w * 256 + c] = acc[q];
  }
  __syncthreads();
  for (int c = tid; c < k; c += kBlock) {
    double sum = red[c];
    for (int ww = 1; ww < kWaves; ++ww) sum += red[ww * 256 + c];
    t[c] = sum;
  }
  __syncthreads();
}

// Q v for a dense Q of one workgroup: full n x n rows (Q.dense = 1), or Q =
// F F' + diag(d) from its factor (Q.dense = 2; Q.rank = k; the block holds F
// (n x k), F' (k x n) and d, row-major, at M): t = F' v into tscr (k), then
// F t + d v, 2 n k values read instead of n^2.
template <typename V, typename Gen, typename Epi>
__device__ void dense_rows(const V* M, const DevMat& Q, double* svec, double* tscr, Gen gen, Epi epi) {
  const int n = Q.nrows;
  if (Q.dense != 2) {
    rect_rows(M, n, n, svec, gen, epi);
    return;
  }
  const int k = Q.rank;
  const V* Ft = M + (int64_t)n * k;
  const V* d = Ft + (int64_t)k * n;
  if (n <= kDenseTile && k <= 256) {
    __syncthreads();
    for (int j = (int)threadIdx.x; j < n; j += kBlock) svec[j] = gen(j, true);
    __syncthreads();
    double* red = tile_lds().prod;  // no tile is staged during a dense product
    if constexpr (sizeof(V) == 4) factor_tv4(M, n, k, svec, red, tscr);
    else if (k <= 64) factor_tv<1>(M, n, k, svec, red, tscr);
    else if (k <= 128) factor_tv<2>(M, n, k, svec, red, tscr);
    else if (k <= 192) factor_tv<3>(M, n, k, svec, red, tscr);
    else factor_tv<4>(M, n, k, svec, red, tscr);
  } else {
    auto put_t = [&](int c, double s) { tscr[c] = s; };
    rect_rows(M, n, k, svec, gen, put_t);  // (ends with a workgroup barrier: tscr visible)
  }
  auto get_t = [&](int c, bool) { return tscr[c]; };
  auto fin = [&](int i, double s) { epi(i, s + (double)d[i] * gen(i, false)); };
  rect_rows(Ft, k, n, svec, get_t, fin);
}

// out = Q xv for a dense Q owned by one workgroup
__device__ __attribute__((noinline)) void dense_qx(const SolveParams& P, const double* xv, double* svec, double* out) {
  dense_rows(P.Q.val, P.Q, svec, P.lr_t, [&](int j, bool) { return xv[j]; }, [&](int i, double v) { out[i] = v; });
}

// CG product for a dense Q owned by one workgroup: stage p in LDS, stream Q
template <typename V>
__device__ __attribute__((noinline)) void dense_cg_spmv(const SolveParams& P, Block B, const V* qd,
                                                        const double* pprev, double* pcur, double beta, int first,
                                                        double inv_tau, double* lds, double* svec) {
  double s[1] = {0.0}, dummy[1] = {0.0};
  dense_rows(
      qd, P.Q, svec, P.lr_t,
      [&](int j, bool first_pass) {
        const double pj = first ? P.r[j] : P.r[j] + beta * pprev[j];
        if (first_pass) pcur[j] = pj;
        return pj;
      },
      [&](int i, double qp) {
        const double pi = first ? P.r[i] : P.r[i] + beta * pprev[i];
        const double qi = qp + pi * inv_tau;
        P.q[i] = qi;
        s[0] += pi * qi;
      });
  block_reduce<1, 0>(s, dummy, lds);
  if (B.tid == 0) P.part[S_PQ * B.nb + B.b] = s[0];
}

// How the n-side pass of a dense Q obtains Q xv: formed into the free CG
// buffer q (the average's evaluation), formed into qx (the current point, which
// then keeps it), or read from qx as kept by the CG updates (no product).
enum QxMode { QX_INTO_Q = 0, QX_FORM = 1, QX_KEPT = 2 };

// n-side product at (xv, yv): g = Q xv + A' yv + c, row by row over the
// workgroup's rows of the partition `pt`.  Writes r = -g (and its FP32 copy)
// when r != null and stores the six n-side partials at slot0.
template <bool DENSE>
__device__ __attribute__((noinline)) void phase_nside(const SolveParams& P, const WgPart& pt, Block B, const double* xv,
                            const double* yv, double* r, float* r32, int r32_stride, int slot0, double* lds,
                            double* svec, int qmode = QX_INTO_Q) {
  // dense Q (one workgroup per QP): Q xv first, into q or qx, unless qx is kept
  constexpr bool dense = DENSE;
  double* const qsrc = qmode == QX_INTO_Q ? P.q : P.qx;
  if (dense && qmode != QX_KEPT) dense_qx(P, xv, svec, qsrc);
  const int G = pt.group;
  double s[3] = {0.0, 0.0, 0.0};   // g.g, x.Qx, c.x
  double mx[3] = {0.0, 0.0, 0.0};  // |g|, |Qx|, |A'y|
  // a low-rank Q gathers t = P' xv (formed by phase_lr_t) and adds d xv below
  GatherVec<double> gx{P.lr_d ? P.lr_pt : xv}, gy{yv};
  auto qxd = [&](int i, double qx, double xi) { return P.lr_d ? qx + gld(P.lr_d + i) * xi : qx; };
  struct Row {
    double c, x, q, d;
  };
  // d = D2_j when the data are preconditioned: the residual maxima are those
  // of the caller's problem, (Qx)_j = (Q~x~)_j / D2_j and likewise A'y and c
  const double* dn = P.dn;
  auto pre = [&](int i) {
    return Row{gld(P.c + i), gld(xv + i), dense ? gld(qsrc + i) : 0.0, dn ? gld(dn + i) : 1.0};
  };
  auto epi = [&](int i, double qx, double aty, const Row& rw) {
    const double g = qx + aty + rw.c;
    if (r) {
      gst(r + i, -g);
      if (r32) gst(r32 + (int64_t)r32_stride * i, (float)(-g));
      if (P.x_prev) gst(P.x_prev + i, rw.x);  // x^k, for the adaptive step's trials
    }
    s[0] += g * g;
    s[1] += rw.x * qx;
    s[2] += rw.c * rw.x;
    if (dn) {
      mx[0] = maxp(mx[0], fabs(g) / rw.d);
      mx[1] = maxp(mx[1], fabs(qx) / rw.d);
      mx[2] = maxp(mx[2], fabs(aty) / rw.d);
    } else {
      mx[0] = maxp(mx[0], fabs(g));
      mx[1] = maxp(mx[1], fabs(qx));
      mx[2] = maxp(mx[2], fabs(aty));
    }
  };
  for (int t = pt.t0; t < pt.t1; ++t)
    tile_rows2(dense ? nullptr : P.Q.rowptr, P.Q.col, P.Q.val, gx, P.m > 0 ? P.At.rowptr : nullptr, P.At.col,
               P.At.val, gy, pt.tile(t), G, pre,
               [&](int i, double qx, double aty, const Row& rw) { epi(i, dense ? rw.q : qxd(i, qx, rw.x), aty, rw); });
  for (int t = pt.l0; t < pt.l1; ++t) {
    const int i = pt.long_rows[t];
    double v[2] = {dense ? 0.0 : row_partial(P.Q.col, P.Q.val, P.Q.rowptr[i], P.Q.rowptr[i + 1], B.tid, kBlock, gx),
                   P.m > 0 ? row_partial(P.At.col, P.At.val, P.At.rowptr[i], P.At.rowptr[i + 1], B.tid, kBlock, gy)
                           : 0.0};
    double dummy[1] = {0.0};
    block_reduce<2, 0>(v, dummy, lds);
    if (B.tid == 0) {
      const Row rw = pre(i);
      epi(i, dense ? rw.q : qxd(i, v[0], rw.x), v[1], rw);
    }
  }
  block_reduce<3, 3>(s, mx, lds);
  if (B.tid == 0) {
    P.part[(slot0 + S_GG) * B.nb + B.b] = s[0];
    P.part[(slot0 + S_XQX) * B.nb + B.b] = s[1];
    P.part[(slot0 + S_CX) * B.nb + B.b] = s[2];
    P.part[(slot0 + S_MG) * B.nb + B.b] = mx[0];
    P.part[(slot0 + S_MQX) * B.nb + B.b] = mx[1];
    P.part[(slot0 + S_MATY) * B.nb + B.b] = mx[2];
  }
}

// m-side product u = A xg over the workgroup's rows of pm, with a per-row
// epilogue epi(i, u) that returns nothing and accumulates the three m-side
// partials (max (u-b)^+, max |u|, sum b.y) through the references given.
template <typename V, typename Tx, typename Pre, typename Epi>
__device__ void mside_rows(const SolveParams& P, Block B, const V* aval, const Tx* xg, double* lds,
                           const Pre& pre, Epi epi) {
  const WgPart& pt = P.w_m;
  GatherVec<Tx> gx{xg};
  const bool res = pt.lcol != nullptr && (int)sizeof(V) == P.res_vbytes;  // rows of A held in LDS
  for (int t = pt.t0; t < pt.t1; ++t) {
    if (res)
      tile_rows_res(pt.lrp, pt.r0, pt.lcol, (const V*)pt.lval, pt.e0, pt.tile(t), pt.group, gx, pre, epi);
    else
      tile_rows_pf(P.A.rowptr, P.A.col, aval, pt.tile(t), pt.group, gx, pre, epi);
  }
  for (int t = pt.l0; t < pt.l1; ++t) {
    const int i = pt.long_rows[t];
    double v[1] = {row_partial(P.A.col, aval, P.A.rowptr[i], P.A.rowptr[i + 1], B.tid, kBlock, gx)};
    double dummy[1] = {0.0};
    block_reduce<1, 0>(v, dummy, lds);
    if (B.tid == 0) epi(i, v[0], pre(i));
  }
}

// per-row inputs of the m-side epilogues (d = D1_i when preconditioned, else 1)
struct MRow {
  double b, y, ax, ya, d;
};

__device__ __forceinline__ double mrow_scale(const SolveParams& P, int i) { return P.dm ? gld(P.dm + i) : 1.0; }

// the m-side maxima (u - b)^+ and |u| of a row, in the caller's units
__device__ __forceinline__ void mside_max(const SolveParams& P, double* mx, double u, const MRow& rw) {
  if (P.dm) {
    mx[0] = maxp(mx[0], pos_part(u - rw.b) / rw.d);
    mx[1] = maxp(mx[1], fabs(u) / rw.d);
  } else {
    mx[0] = maxp(mx[0], pos_part(u - rw.b));
    mx[1] = maxp(mx[1], fabs(u));
  }
}

__device__ void store_mside(const SolveParams& P, Block B, int slot0, double* s1, double* mx, double* lds) {
  block_reduce<1, 2>(s1, mx, lds);
  if (B.tid == 0) {
    P.part[(slot0 + S_MVIOL) * B.nb + B.b] = mx[0];
    P.part[(slot0 + S_MAX) * B.nb + B.b] = mx[1];
    P.part[(slot0 + S_BY) * B.nb + B.b] = s1[0];
  }
}

// ax = A x and the m-side partials of the current point (start of a solve)
__device__ __attribute__((noinline)) void phase_ax(const SolveParams& P, Block B, double* lds) {
  double s1[1] = {0.0}, mx[2] = {0.0, 0.0};
  mside_rows(
      P, B, P.A.val, P.x, lds, [&](int i) { return MRow{gld(P.b + i), gld(P.y + i), 0.0, 0.0, mrow_scale(P, i)}; },
      [&](int i, double u, const MRow& rw) {
        gst(P.ax + i, u);
        mside_max(P, mx, u, rw);
        s1[0] += rw.b * rw.y;
      });
  store_mside(P, B, 0, s1, mx, lds);
}

// relKKT pieces of the average: n-side at (xa, ya), m-side u = A xa (kept in ax_avg)
template <bool DENSE>
__device__ __attribute__((noinline)) void phase_eval_avg(const SolveParams& P, Block B, double* lds, double* svec) {
  phase_nside<DENSE>(P, P.w_n1, B, P.xa, P.ya, nullptr, nullptr, 1, S_AVG0, lds, svec);
  double s1[1] = {0.0}, mx[2] = {0.0, 0.0};
  mside_rows(
      P, B, P.A.val, P.xa, lds, [&](int i) { return MRow{gld(P.b + i), 0.0, 0.0, gld(P.ya + i), mrow_scale(P, i)}; },
      [&](int i, double u, const MRow& rw) {
        gst(P.ax_avg + i, u);
        mside_max(P, mx, u, rw);
        s1[0] += rw.b * rw.ya;
      });
  store_mside(P, B, S_AVG0, s1, mx, lds);
}

// CG product: p = r + beta p_prev on the owned rows (FP64, stored), and
// q = (Q + I/tau) p with p gathered through gp (GatherDir on the FP64 r and
// p_prev, or GatherDir2 on the FP32 (r, p) records); partial p.q.
template <bool DENSE, typename V, typename G>
__device__ __attribute__((noinline)) void phase_cg_spmv(const SolveParams& P, Block B, const V* qval, const G gp,
                              const double* pprev, double* pcur, double beta, int first,
                              double inv_tau, double* lds, double* svec) {
  if constexpr (DENSE) {
    dense_cg_spmv(P, B, qval, pprev, pcur, beta, first, inv_tau, lds, svec);
    return;
  }
  const WgPart& pt = P.w_cg;
  double s[1] = {0.0};
  using T = std::conditional_t<sizeof(V) == 4, float, double>;  // gathered t: FP32 with FP32 values
  if (P.lr_d) {  // low-rank Q: (P t)_i with t = P' p gathered, then + (d_i + 1/tau) p_i
    const T* tv;
    if constexpr (sizeof(V) == 4) tv = (const T*)P.lr_pt32; else tv = (const T*)P.lr_pt;
    const GatherVec<T> gt{tv};
    auto epi = [&](int i, double pt_i) {
      const double pi = first ? P.r[i] : P.r[i] + beta * pprev[i];
      const double qi = pt_i + (gld(P.lr_d + i) + inv_tau) * pi;
      pcur[i] = pi;
      P.q[i] = qi;
      s[0] += pi * qi;
    };
    for (int t = pt.t0; t < pt.t1; ++t) tile_rows(P.Q.rowptr, P.Q.col, qval, pt.tile(t), pt.group, gt, epi);
    for (int t = pt.l0; t < pt.l1; ++t) {
      const int i = pt.long_rows[t];
      double v[1] = {row_partial(P.Q.col, qval, P.Q.rowptr[i], P.Q.rowptr[i + 1], B.tid, kBlock, gt)};
      double dummy[1] = {0.0};
      block_reduce<1, 0>(v, dummy, lds);
      if (B.tid == 0) epi(i, v[0]);
    }
    double dummy[1] = {0.0};
    block_reduce<1, 0>(s, dummy, lds);
    if (B.tid == 0) P.part[S_PQ * B.nb + B.b] = s[0];
    return;
  }
  auto epi = [&](int i, double qp) {
    const double pi = first ? P.r[i] : P.r[i] + beta * pprev[i];
    const double qi = qp + pi * inv_tau;
    pcur[i] = pi;
    P.q[i] = qi;
    s[0] += pi * qi;
  };
  for (int t = pt.t0; t < pt.t1; ++t) tile_rows(P.Q.rowptr, P.Q.col, qval, pt.tile(t), pt.group, gp, epi);
  for (int t = pt.l0; t < pt.l1; ++t) {
    const int i = pt.long_rows[t];
    double v[1] = {row_partial(P.Q.col, qval, P.Q.rowptr[i], P.Q.rowptr[i + 1], B.tid, kBlock, gp)};
    double dummy[1] = {0.0};
    block_reduce<1, 0>(v, dummy, lds);
    if (B.tid == 0) epi(i, v[0]);
  }
  double dummy[1] = {0.0};
  block_reduce<1, 0>(s, dummy, lds);
  if (B.tid == 0) P.part[S_PQ * B.nb + B.b] = s[0];
}

// t = P' v for a low-rank Q = P P' + diag(d): the rows of P' in the
// workgroup's share of plr, v gathered through g (x or the average for the
// n-side pass, the direction p = r + beta p_prev formed at gather time for a
// CG product); t goes to lr_pt and its FP32 copy to lr_pt32.  No partials.
template <typename V, typename G>
__device__ __attribute__((noinline)) void phase_lr_t(const SolveParams& P, Block B, const V* lval, const G g,
                                                     double* lds) {
  const WgPart& pt = P.w_lr;
  auto epi = [&](int c, double t) {
    P.lr_pt[c] = t;
    P.lr_pt32[c] = (float)t;
  };
  for (int t = pt.t0; t < pt.t1; ++t) tile_rows(P.Lt.rowptr, P.Lt.col, lval, pt.tile(t), pt.group, g, epi);
  for (int t = pt.l0; t < pt.l1; ++t) {
    const int c = pt.long_rows[t];
    double v[1] = {row_partial(P.Lt.col, lval, P.Lt.rowptr[c], P.Lt.rowptr[c + 1], B.tid, kBlock, g)};
    double dummy[1] = {0.0};
    block_reduce<1, 0>(v, dummy, lds);
    if (B.tid == 0) epi(c, v[0]);
  }
}

// CG update on the owned rows: x += alpha p, r -= alpha q; partial r.r.
// With qx kept (a dense Q in the batch), Q x moves with x by linearity:
// Q x += alpha Q p, Q p = q - p / tau.
__device__ __attribute__((noinline)) void phase_cg_update(const SolveParams& P, Block B, const double* pcur, double alpha, int mixed,
                                double inv_tau, double* lds) {
  const int r0 = P.w_cg.r0, r1 = P.w_cg.r1;
  double s[1] = {0.0};
  double* const qx = P.qx;
  for (int i = r0 + B.tid; i < r1; i += kBlock) {
    const double pi = pcur[i], qi = P.q[i];
    const double xi = P.x[i] + alpha * pi;
    const double ri = P.r[i] - alpha * qi;
    if (qx) qx[i] += alpha * (qi - pi * inv_tau);
    P.x[i] = xi;
    P.r[i] = ri;
    if (mixed) {
      P.x32[i] = (float)xi;
      gst2(P.rp32 + i, (float)ri, (float)pi);  // the next product's (r, p_prev)
    }
    s[0] += ri * ri;
  }
  double dummy[1] = {0.0};
  block_reduce<1, 0>(s, dummy, lds);
  if (B.tid == 0) P.part[S_RR * B.nb + B.b] = s[0];
}

// One step of CG in the single-reduction form of Chronopoulos and Gear, as
// one phase.  With u = (Q + I/tau) r and s = (Q + I/tau) p kept alongside
// r and p, step l (l >= 1, given alpha = alpha_{l-1}, beta = beta_{l-1})
// forms on the owned rows
//   s_{l-1} = u_{l-1} + beta s_{l-2},  p_{l-1} = r_{l-1} + beta p_{l-2},
//   x += alpha p_{l-1},  r_l = r_{l-1} - alpha s_{l-1},
// and u_l = (Q + I/tau) r_l with r_l formed at gather time from r_{l-1},
// u_{l-1}, s_{l-2} of the other rows; the partials gamma_l = r_l.r_l and
// delta_l = r_l.u_l then give beta_l = gamma_l / gamma_{l-1} and
// alpha_l = gamma_l / (delta_l - beta_l gamma_l / alpha_{l-1}).  In exact
// arithmetic this is the same iteration as the textbook CG of the primal step
// (same x, r, step lengths), with one grid barrier per step instead of two.
// Step 0 only forms u_0 = (Q + I/tau) r_0 and delta_0.  With product = false
// (the last allowed step) only x is advanced.
template <typename T>
struct GatherCG {
  const T* r;
  const T* u;
  const T* s;
  double alpha, beta;
  int l;
  // unconditional loads (u and s are always valid buffers; values not used
  // at the current step are discarded by the selects), so that a tile's
  // gathers all issue before the first wait
  __device__ __forceinline__ double operator()(int j) const {
    const double rj = (double)gld(r + j), uj = (double)gld(u + j), sj = (double)gld(s + j);
    const double s1 = l == 1 ? uj : uj + beta * sj;
    return l == 0 ? rj : rj - alpha * s1;
  }
};

// the same with the FP32 copies of (r, u, s) interleaved per row: one
// 16-byte load per gathered column instead of three loads on three lines
struct GatherCG4 {
  const float4* v;
  double alpha, beta;
  int l;
  __device__ __forceinline__ double operator()(int j) const {
    const float4 q = gld(v + j);
    const double rj = q.x, uj = q.y, sj = q.z;
    const double s1 = l == 1 ? uj : uj + beta * sj;
    return l == 0 ? rj : rj - alpha * s1;
  }
};

// Buffers: r, u, s (FP64, and in mixed precision their FP32 copies
// interleaved as float4 rows) alternate between two copies.  Step l reads
// copy rd = (l == 0 ? 0 : 1 - l mod 2) and writes copy c = l mod 2: r_l and
// u_l, and s_{l-1}, which step l + 1 reads as its s_{l-2}.  The n-side pass
// leaves r_0 in copy 0; step 0 reads it there and adds u_0 (no step reads a
// field another workgroup is writing in the same phase).
//
// When the launch holds the CG state of the workgroup's rows in LDS
// (P.cg_own), x, p, r, u and s of the owned rows live there from step 0 to the
// dual step; device memory then receives only what other workgroups read
// during the primal step: the FP32 x (for the dual product) and the
// interleaved (r, u, s) rows in mixed precision, or x, r, u, s in FP64.  The
// FP64 x of mixed precision is written back by the dual step (phase_dual).
template <typename V, typename T, bool OWN>
__device__ __attribute__((noinline)) void phase_cgcg(const SolveParams& P, Block B, const V* qval, int l,
                                                     double alpha, double beta, double inv_tau, int product,
                                                     int mixed, double* lds) {
  const int c = l & 1;
  const int rd = l == 0 ? 0 : c ^ 1;
  const double* r_prev = rd ? P.r_alt : P.r;
  const double* u_prev = rd ? P.u1 : P.u0;
  const double* s_prev2 = rd ? P.s1 : P.s0;
  double* r_new = c ? P.r_alt : P.r;
  double* u_new = c ? P.u1 : P.u0;
  double* s_prev1 = c ? P.s1 : P.s0;
  float4* v_new = c ? P.v32_1 : P.v32_0;
  double s[2] = {0.0, 0.0};  // gamma_l, delta_l
  // owned-row state in LDS (OWN): x, p, r, u, s at ob + {0, 1, 2, 3, 4} * no
  double* const ob = P.cg_own;
  const int ro0 = P.w_cg.r0, no = P.w_cg.r1 - P.w_cg.r0;
  const bool pub = !OWN || !mixed;  // FP64 r, u, s, x go to device memory
  struct Row {
    double rp, up, sp, pp, xp;
  };
  // the owned-row inputs, loaded unconditionally (all buffers are valid;
  // values not used at this step are discarded by selects)
  // (with the state in LDS only step 0 prefetches: r_0 and x from device
  // memory; later steps read LDS in the epilogue)
  auto pre = [&](int i) {
    if (!OWN) return Row{gld(r_prev + i), gld(u_prev + i), gld(s_prev2 + i), gld(P.p0 + i), gld(P.x + i)};
    if (l == 0) return Row{gld(r_prev + i), 0.0, 0.0, 0.0, gld(P.x + i)};
    return Row{0.0, 0.0, 0.0, 0.0, 0.0};
  };
  struct Own {
    double r, s;  // r_l[i] and s_{l-1}[i]
  };
  auto own = [&](int i, const Row& rw) -> Own {  // owned-row updates
    double rp = rw.rp, up = rw.up, sp = rw.sp, pp = rw.pp, xp = rw.xp;
    double* const o = ob + (i - ro0);
    if (OWN && l > 0) {
      xp = lld(o);
      pp = lld(o + no);
      rp = lld(o + 2 * no);
      up = lld(o + 3 * no);
      sp = lld(o + 4 * no);
    }
    if (l == 0) {
      if (OWN) {
        lst(o, xp);
        lst(o + 2 * no, rp);
      }
      return Own{rp, 0.0};
    }
    const double s1 = l == 1 ? up : up + beta * sp;
    const double pi = l == 1 ? rp : rp + beta * pp;
    const double xi = xp + alpha * pi;
    if (OWN) {
      lst(o + no, pi);
      lst(o, xi);
    } else {
      gst(P.p0 + i, pi);
    }
    if (pub) gst(P.x + i, xi);
    if (mixed) gst(P.x32 + i, (float)xi);
    if (!product) return Own{0.0, 0.0};
    const double ri = rp - alpha * s1;
    if (OWN) {
      lst(o + 4 * no, s1);
      lst(o + 2 * no, ri);
    }
    if (pub) {
      gst(s_prev1 + i, s1);
      gst(r_new + i, ri);
    }
    return Own{ri, s1};
  };
  if (!product) {
    for (int i = ro0 + B.tid; i < ro0 + no; i += kBlock) own(i, pre(i));
    return;
  }
  auto epi = [&](int i, double qr, const Row& rw) {
    const Own ow = own(i, rw);
    const double ui = qr + ow.r * inv_tau;
    if (OWN) lst(ob + (i - ro0) + 3 * no, ui);
    if (pub) gst(u_new + i, ui);
    if (mixed) gst(v_new + i, make_float4((float)ow.r, (float)ui, (float)ow.s, 0.0f));
    s[0] += ow.r * ow.r;
    s[1] += ow.r * ui;
  };
  const WgPart& pt = P.w_cg;
  const bool res = pt.lcol != nullptr && (int)sizeof(V) == P.res_vbytes;  // rows of Q held in LDS
  auto run = [&](const auto& g) {
    for (int t = pt.t0; t < pt.t1; ++t) {
      if (res)
        tile_rows_res(pt.lrp, pt.r0, pt.lcol, (const V*)pt.lval, pt.e0, pt.tile(t), pt.group, g, pre, epi);
      else
        tile_rows_pf(P.Q.rowptr, P.Q.col, qval, pt.tile(t), pt.group, g, pre, epi);
    }
    for (int t = pt.l0; t < pt.l1; ++t) {
      const int i = pt.long_rows[t];
      double v[1] = {row_partial(P.Q.col, qval, P.Q.rowptr[i], P.Q.rowptr[i + 1], B.tid, kBlock, g)};
      double dummy[1] = {0.0};
      block_reduce<1, 0>(v, dummy, lds);
      if (B.tid == 0) epi(i, v[0], pre(i));
    }
  };
  if constexpr (std::is_same<T, float>::value)
    run(GatherCG4{rd ? P.v32_1 : P.v32_0, alpha, beta, l});
  else
    run(GatherCG<double>{r_prev, u_prev, s_prev2, alpha, beta, l});
  double dummy[1] = {0.0};
  block_reduce<2, 0>(s, dummy, lds);
  if (B.tid == 0) {
    P.part[S_RR * B.nb + B.b] = s[0];
    P.part[S_PQ * B.nb + B.b] = s[1];
  }
}

// Dual step and averages (Alg. 1): u = A x^{k+1};
// y <- max(0, y + sigma (2u - A x^k - b)); A x^k <- u; ya += w (y - ya);
// xa += w (x - xa) on an n-slice; m-side partials of the new point.
// xo: the LDS x of the CG rows when the primal step kept it there (null:
// device memory holds x); in mixed precision it is written back here.
template <typename V, typename Tx>
__device__ __attribute__((noinline)) void phase_dual(const SolveParams& P, Block B, const V* aval, const Tx* xg,
                                                     double sigma, double w, const double* xo, double* lds) {
  double s1[1] = {0.0}, mx[2] = {0.0, 0.0};
  mside_rows(
      P, B, aval, xg, lds,
      [&](int i) { return MRow{gld(P.b + i), gld(P.y + i), gld(P.ax + i), gld(P.ya + i), mrow_scale(P, i)}; },
      [&](int i, double u, const MRow& rw) {
        const double yn = pos_part(rw.y + sigma * (2.0 * u - rw.ax - rw.b));
        gst(P.y + i, yn);
        gst(P.ax + i, u);
        gst(P.ya + i, rw.ya + w * (yn - rw.ya));
        mside_max(P, mx, u, rw);
        s1[0] += rw.b * yn;
      });
  const int r0 = P.w_cg.r0, r1 = P.w_cg.r1;
  for (int j = r0 + B.tid; j < r1; j += kBlock) {
    const double xaj = gld(P.xa + j);
    double xj;
    if (xo) {
      xj = lld(xo + (j - r0));
      if (sizeof(Tx) == 4) gst(P.x + j, xj);  // (in FP64 the primal step already wrote it)
    } else {
      xj = gld(P.x + j);
    }
    gst(P.xa + j, xaj + w * (xj - xaj));
  }
  store_mside(P, B, 0, s1, mx, lds);
}

// Adaptive step size (Sec. 4): the dual step of a trial, kept apart from the
// iterate until the trial is accepted.  u = A x', y' = max(0, y + sigma (2u -
// Ax - b)) go to y_trial and ax_trial, the m-side partials of (x', y') to the
// trial slots, and the pieces of the trial's step limit to theirs:
// ||dy||^2 and dy.(A dx) = dy.(u - Ax) over the m rows, ||dx||^2 and
// dx.(Q dx) over the CG rows, with dx = x' - x^k gathered in FP64 and Q's
// FP64 values.
struct GatherDiff {
  const double* a;
  const double* b;
  __device__ __forceinline__ double operator()(int j) const { return gld(a + j) - gld(b + j); }
};

template <bool DENSE, typename V, typename Tx>
__device__ __attribute__((noinline)) void phase_dual_trial(const SolveParams& P, Block B, const V* aval,
                                                           const Tx* xg, double sigma, double* lds, double* svec) {
  double sm[5] = {0.0, 0.0, 0.0, 0.0, 0.0};  // b.y', dy.dy, dy.(u - Ax), dx.dx, dx.(Q dx)
  double mx[2] = {0.0, 0.0};
  mside_rows(
      P, B, aval, xg, lds,
      [&](int i) { return MRow{gld(P.b + i), gld(P.y + i), gld(P.ax + i), 0.0, mrow_scale(P, i)}; },
      [&](int i, double u, const MRow& rw) {
        const double yn = pos_part(rw.y + sigma * (2.0 * u - rw.ax - rw.b));
        gst(P.y_trial + i, yn);
        gst(P.ax_trial + i, u);
        mside_max(P, mx, u, rw);
        const double dy = yn - rw.y;
        sm[0] += rw.b * yn;
        sm[1] += dy * dy;
        sm[2] += dy * (u - rw.ax);
      });
  auto epi = [&](int i, double qd) {
    const double dx = gld(P.x + i) - gld(P.x_prev + i);
    sm[3] += dx * dx;
    sm[4] += dx * qd;
  };
  if constexpr (DENSE) {
    dense_rows(P.Q.val, P.Q, svec, P.lr_t, [&](int j, bool) { return gld(P.x + j) - gld(P.x_prev + j); }, epi);
  } else {
    const WgPart& pt = P.w_cg;
    const GatherDiff g{P.x, P.x_prev};
    for (int t = pt.t0; t < pt.t1; ++t) tile_rows(P.Q.rowptr, P.Q.col, P.Q.val, pt.tile(t), pt.group, g, epi);
    for (int t = pt.l0; t < pt.l1; ++t) {
      const int i = pt.long_rows[t];
      double v[1] = {row_partial(P.Q.col, P.Q.val, P.Q.rowptr[i], P.Q.rowptr[i + 1], B.tid, kBlock, g)};
      double dummy[1] = {0.0};
      block_reduce<1, 0>(v, dummy, lds);
      if (B.tid == 0) epi(i, v[0]);
    }
  }
  block_reduce<5, 2>(sm, mx, lds);
  if (B.tid == 0) {
    P.part[S_TBY * B.nb + B.b] = sm[0];
    P.part[S_DY2 * B.nb + B.b] = sm[1];
    P.part[S_DYADX * B.nb + B.b] = sm[2];
    P.part[S_DX2 * B.nb + B.b] = sm[3];
    P.part[S_DXQDX * B.nb + B.b] = sm[4];
    P.part[S_TVIOL * B.nb + B.b] = mx[0];
    P.part[S_TMAX * B.nb + B.b] = mx[1];
  }
}

// An accepted trial becomes the iterate: y = y', Ax = A x', the averages take
// it with weight w (Alg. 1), and the trial's m-side partials become those of
// the current point (each workgroup moves its own).
__device__ __attribute__((noinline)) void phase_commit(const SolveParams& P, Block B, double w) {
  const int m0 = P.w_m.r0, m1 = P.w_m.r1;
  for (int i = m0 + B.tid; i < m1; i += kBlock) {
    const double yn = gld(P.y_trial + i), ya = gld(P.ya + i);
    gst(P.y + i, yn);
    gst(P.ax + i, gld(P.ax_trial + i));
    gst(P.ya + i, ya + w * (yn - ya));
  }
  const int n0 = P.w_cg.r0, n1 = P.w_cg.r1;
  for (int j = n0 + B.tid; j < n1; j += kBlock) {
    const double xa = gld(P.xa + j);
    gst(P.xa + j, xa + w * (gld(P.x + j) - xa));
  }
  if (B.tid == 0) {
    P.part[S_MVIOL * B.nb + B.b] = P.part[S_TVIOL * B.nb + B.b];
    P.part[S_MAX * B.nb + B.b] = P.part[S_TMAX * B.nb + B.b];
    P.part[S_BY * B.nb + B.b] = P.part[S_TBY * B.nb + B.b];
  }
}

// A rejected trial: back to x^k (y and Ax were left as they were).
__device__ __attribute__((noinline)) void phase_retry(const SolveParams& P, Block B) {
  const int n0 = P.w_cg.r0, n1 = P.w_cg.r1;
  for (int j = n0 + B.tid; j < n1; j += kBlock) {
    const double xk = gld(P.x_prev + j);
    gst(P.x + j, xk);
    if (P.x32) gst(P.x32 + j, (float)xk);
  }
}

// Restart: move to the candidate (average when use_avg), measure the
// movement from the previous anchor, and make the candidate the new anchor
// and the new (empty) average.
__device__ __attribute__((noinline)) void phase_restart(const SolveParams& P, Block B, int use_avg, int mixed, double* lds) {
  double s[2] = {0.0, 0.0};
  const int n0 = P.w_cg.r0, n1 = P.w_cg.r1;
  for (int j = n0 + B.tid; j < n1; j += kBlock) {
    const double xc = use_avg ? P.xa[j] : P.x[j];
    const double d = xc - P.x_anc[j];
    s[0] += d * d;
    P.x[j] = xc;
    if (mixed) P.x32[j] = (float)xc;
    P.x_anc[j] = xc;
    P.xa[j] = xc;
  }
  const int m0 = P.w_m.r0, m1 = P.w_m.r1;
  for (int i = m0 + B.tid; i < m1; i += kBlock) {
    const double yc = use_avg ? P.ya[i] : P.y[i];
    const double d = yc - P.y_anc[i];
    s[1] += d * d;
    P.y[i] = yc;
    P.y_anc[i] = yc;
    P.ya[i] = yc;
    if (use_avg) P.ax[i] = P.ax_avg[i];
  }
  double dummy[1] = {0.0};
  block_reduce<2, 0>(s, dummy, lds);
  if (B.tid == 0) {
    P.part[S_DX * B.nb + B.b] = s[0];
    P.part[S_DY * B.nb + B.b] = s[1];
    if (use_avg) {
      P.part[S_MVIOL * B.nb + B.b] = P.part[(S_AVG0 + S_MVIOL) * B.nb + B.b];
      P.part[S_MAX * B.nb + B.b] = P.part[(S_AVG0 + S_MAX) * B.nb + B.b];
      P.part[S_BY * B.nb + B.b] = P.part[(S_AVG0 + S_BY) * B.nb + B.b];
    }
  }
}

// copy src -> dst on the workgroup's n- and m-slices (returning the average
// or restoring the anchor at the end of a solve)
__device__ __attribute__((noinline)) void phase_copy_point(const SolveParams& P, Block B, const double* xs, const double* ys) {
  const int n0 = P.w_cg.r0, n1 = P.w_cg.r1;
  for (int j = n0 + B.tid; j < n1; j += kBlock) P.x[j] = xs[j];
  const int m0 = P.w_m.r0, m1 = P.w_m.r1;
  for (int i = m0 + B.tid; i < m1; i += kBlock) P.y[i] = ys[i];
}

// x, y, their averages and anchors, Ax and the FP32 copy of x set to zero
__device__ __attribute__((noinline)) void phase_zero_point(const SolveParams& P, Block B) {
  const int n0 = P.w_cg.r0, n1 = P.w_cg.r1;
  for (int j = n0 + B.tid; j < n1; j += kBlock) {
    P.x[j] = 0.0;
    P.xa[j] = 0.0;
    P.x_anc[j] = 0.0;
    if (P.x32) P.x32[j] = 0.0f;
  }
  const int m0 = P.w_m.r0, m1 = P.w_m.r1;
  for (int i = m0 + B.tid; i < m1; i += kBlock) {
    P.y[i] = 0.0;
    P.ya[i] = 0.0;
    P.y_anc[i] = 0.0;
  }
}

// relKKT (Sec. 4, progress metric) from the reduced partials of one point.
struct Kkt {
  double rp, rd, rg, kkt, pobj, dobj;
};

__device__ Kkt kkt_from(const double* s, const double* mx, double nb_inf, double nc_inf) {
  // s: g.g, x.Qx, c.x, b.y ; mx: |g|, |Qx|, |A'y|, (u-b)^+, |u|
  Kkt k;
  const double xqx = s[1], cx = s[2], by = s[3];
  k.rp = rel_div(mx[3], maxp(mx[4], nb_inf));
  k.rd = rel_div(mx[0], maxp(mx[1], maxp(mx[2], nc_inf)));
  k.rg = fabs(xqx + cx + by) / (1.0 + maxp(fabs(0.5 * xqx + cx), fabs(0.5 * xqx + by)));
  k.kkt = maxp(k.rp, maxp(k.rd, k.rg));
  k.pobj = 0.5 * xqx + cx;
  k.dobj = -0.5 * xqx - by;
  return k;
}

// relKKT pieces from the partials at slot0 (and, when gg / flag are given,
// g.g and the time-limit flag); thread 0 writes them to *out, *gg, *flag (LDS)
__device__ __attribute__((noinline)) void reduce_kkt(const SolveParams& P, Block B, int slot0, double nb_inf,
                                                     double nc_inf, Kkt* out, double* gg, double* flag,
                                                     double* lds) {
  const int ss[4] = {slot0 + S_GG, slot0 + S_XQX, slot0 + S_CX, slot0 + S_BY};
  const int ms[6] = {slot0 + S_MG, slot0 + S_MQX, slot0 + S_MATY, slot0 + S_MVIOL, slot0 + S_MAX, S_FLAG};
  double s[4], mx[6];
  reduce_partials<4, 6>(P.part, B.nb, ss, ms, s, mx, lds);
  if (B.tid == 0) {
    if (gg) *gg = s[0];
    if (flag) *flag = mx[5];
    Kkt k = kkt_from(s, mx, nb_inf, nc_inf);
    // a NaN anywhere in g shows in g.g even where the max would not see it
    if (!(s[0] == s[0])) k.kkt = s[0];
    *out = k;
  }
}

__device__ __attribute__((noinline)) double reduce_one(const SolveParams& P, Block B, int slot, double* lds) {
  const int ss[1] = {slot};
  const int ms[1] = {0};
  double s[1], mx[1];
  reduce_partials<1, 0>(P.part, B.nb, ss, ms, s, mx, lds);
  return s[0];
}



// ------------------------------------------------------------- main kernel

// The restarted PDHCG loop (Alg. 1 with the practical rules of Sec. 4),
// shared by the cooperative single-QP kernel (many workgroups, grid
// barriers) and the batched kernel (one workgroup per QP, nb = 1, where a
// barrier is a workgroup barrier).
//
// Every thread of the workgroup runs the data-parallel phases and the
// reductions of their partials; the scalar logic (relKKT tests, restart
// rules, step sizes, CG coefficients) runs on one control thread that keeps
// the solver state in LDS and writes the next phase and its arguments there.
// The state thus occupies no vector registers across phases, and every
// workgroup's control thread takes the same decisions from the same reduced
// values.

// phases the control thread can schedule
enum Op : int32_t {
  OP_END = 0,
  OP_AX_START,     // m-side of the start point (first launch of a solve)
  OP_NSIDE,        // n-side pass at the current point, relKKT pieces
  OP_ZERO,         // warm-start fallback: the start point is replaced by (0, 0)
  OP_AX_ZERO,      // ... and its m-side recomputed
  OP_CERTIFY,      // FP64 m-side of a point that passed with FP32 products
  OP_EVAL,         // relKKT of the running average
  OP_RESTART,      // restart to the candidate
  OP_LIMIT_AX,     // exact m-side before reporting at a limit
  OP_LIMIT_EVAL,   // average's relKKT before reporting at a limit
  OP_CG,           // one step of single-reduction CG
  OP_CG_SPMV,      // textbook CG: product
  OP_CG_UPDATE,    // textbook CG: update
  OP_DUAL,         // dual step and averages
  OP_COPY_AVG,     // return the average (no barrier follows)
  OP_COPY_ANCHOR,  // return the epoch's anchor (no barrier follows)
  OP_DUAL_TRIAL,   // adaptive step size: dual step of a trial and its step limit
  OP_COMMIT,       // adaptive step size: the accepted trial becomes the iterate
  OP_RETRY,        // adaptive step size: a rejected trial, back to x^k
};

struct Ctl {
  SolverState S;
  Kkt kc, ka;         // relKKT pieces of the current point and of the average
  Kkt rk;             // result of the reduction that followed the last phase
  double ra, rb;      // (its scalar results)
  double rho, tflag;  // r0.r0 of the primal step, time-limit flag
  double Kc;          // candidate relKKT of the pending restart
  double gamma, alpha, beta, inv_tau, w;
  int64_t budget;     // iterations left in this launch
  int32_t op, l, steps, have_avg, use_avg, first, cur;
  int32_t xlds;       // the primal step left x of the CG rows in LDS (P.cg_own)
  int32_t retry;      // the n-side pass repeats x^k's for a rejected trial
  // kept Q x (P.qx): the next n-side pass forms Q x with a product (exact),
  // and whether the current point's relKKT pieces (kc) came from such a pass
  int32_t exact, kc_exact;
  double rt[4];       // sums of a trial: dx.dx, dy.dy, dy.(A dx), dx.(Q dx)
};

__device__ void ctl_end_cg(const SolveParams& P, Ctl& C) {
  C.S.cg_total += C.steps;
  C.w = 1.0 / (double)(C.S.k + 1);  // averages with weight 1/(k+1)
  C.op = P.step_rule ? OP_DUAL_TRIAL : OP_DUAL;
}

// primal step: inexact CG on (Q + I/tau) x = x^k/tau - c - A'y^k (Alg. 1);
// the CG tolerance grows once per iteration (not again for a repeated trial)
__device__ void ctl_start_cg(const SolveParams& P, Ctl& C, bool grow_eps = true) {
  if (grow_eps) C.S.eps += P.eps_factor * C.kc.kkt;
  C.inv_tau = 1.0 / C.S.tau;
  C.steps = 0;
  C.xlds = 0;
  if (C.rho > 0.0 && P.u0 != nullptr) {  // single-reduction CG: L steps take L + 1 grid barriers
    C.xlds = P.cg_own != nullptr;
    C.gamma = C.rho;
    C.alpha = 0.0;
    C.beta = 0.0;
    C.l = 0;
    C.op = OP_CG;
  } else if (C.rho > 0.0) {
    C.beta = 0.0;
    C.first = 1;
    C.cur = 0;
    C.l = 1;
    C.op = OP_CG_SPMV;
  } else {
    ctl_end_cg(P, C);
  }
}

__device__ void ctl_finish(Ctl& C, const Kkt& k, int status, int avg) {
  C.S.done = 1;
  C.S.status = status;
  C.S.returned_average = avg;
  C.S.r_p = k.rp;
  C.S.r_d = k.rd;
  C.S.r_g = k.rg;
  C.S.kkt = k.kkt;
  C.S.pobj = k.pobj;
  C.S.dobj = k.dobj;
}

// at the iteration cap or the time limit: report the better of current and average
__device__ void ctl_limit_report(const SolveParams& P, Ctl& C) {
  const bool at_cap = C.S.k_total >= P.max_iters;
  const bool avg = C.have_avg && C.ka.kkt < C.kc.kkt;
  const Kkt& k = avg ? C.ka : C.kc;
  ctl_finish(C, k, k.kkt <= P.tol ? 0 : (at_cap ? 1 : 2), avg ? 1 : 0);
  C.op = avg ? OP_COPY_AVG : OP_END;
}

__device__ void ctl_limit_after_ax(const SolveParams& P, Ctl& C) {
  if (C.S.k > 0 && !C.have_avg) {
    C.op = OP_LIMIT_EVAL;
    return;
  }
  ctl_limit_report(P, C);
}

__device__ void ctl_limits(const SolveParams& P, Ctl& C) {
  const bool at_cap = C.S.k_total >= P.max_iters;
  const bool at_time = C.tflag > 0.0;
  if (at_cap || at_time) {
    if (P.qx && !C.kc_exact) {  // the reported relKKT from a formed Q x
      C.exact = 1;
      C.op = OP_NSIDE;
      return;
    }
    if (C.S.mixed) {  // exact FP64 m-side partials for the reported relKKT
      C.op = OP_LIMIT_AX;
      return;
    }
    ctl_limit_after_ax(P, C);
    return;
  }
  ctl_start_cg(P, C);
}

// restart evaluation (Sec. 4, adaptive restart) once the average's relKKT is known
__device__ void ctl_after_eval(const SolveParams& P, Ctl& C) {
  C.have_avg = 1;
  C.S.evals += 1;
  if (C.ka.kkt <= P.tol) {
    ctl_finish(C, C.ka, 0, 1);
    C.op = OP_COPY_AVG;
    return;
  }
  const int use_avg = (P.restart_to == 1) || (C.ka.kkt < C.kc.kkt);
  const double Kc = use_avg ? C.ka.kkt : C.kc.kkt;
  int why = 0;
  if (Kc <= P.beta_suf * C.S.K_anchor) why = 1;
  else if (Kc <= P.beta_nec * C.S.K_anchor && Kc > C.S.K_prev) why = 2;
  else if ((double)C.S.k >= P.beta_art * (double)C.S.k_total) why = 3;
  C.S.K_prev = Kc;
  if (why) {
    C.use_avg = use_avg;
    C.Kc = Kc;
    C.op = OP_RESTART;
    return;
  }
  ctl_limits(P, C);
}

// after the current point's relKKT is final (certified when it came from FP32 products)
__device__ void ctl_after_kkt(const SolveParams& P, Ctl& C) {
  if (C.kc.kkt <= P.tol) {
    ctl_finish(C, C.kc, 0, 0);
    C.op = OP_END;
    return;
  }
  if (C.S.k > 0 && C.S.k % P.eval_period == 0) {
    C.op = OP_EVAL;
    return;
  }
  ctl_limits(P, C);
}

__device__ void ctl_after_nside(const SolveParams& P, Ctl& C) {
  C.have_avg = 0;
  if (!C.S.start_checked) {
    C.S.start_checked = 1;
    if (P.kkt_zero > 0.0 && !(C.kc.kkt <= P.kkt_zero)) {  // the given start point is worse than (0, 0)
      C.op = OP_ZERO;
      return;
    }
  }
  if (C.S.K_anchor != C.S.K_anchor) C.S.K_anchor = C.kc.kkt;
  if (!(C.kc.kkt == C.kc.kkt) || isinf(C.kc.kkt)) {  // NUMERICAL_ERROR: back to the anchor
    C.S.done = 1;
    C.S.status = 3;
    C.S.r_p = C.S.r_d = C.S.r_g = NAN;
    C.S.kkt = C.kc.kkt;
    C.S.pobj = C.S.dobj = NAN;
    C.op = OP_COPY_ANCHOR;
    return;
  }
  if (C.kc.kkt <= P.tol && P.qx && !C.kc_exact) {  // Q x was the kept one: form it before stopping
    C.exact = 1;
    C.op = OP_NSIDE;
    return;
  }
  if (C.kc.kkt <= P.tol && C.S.mixed) {  // the m-side partials came from FP32 products
    C.op = OP_CERTIFY;
    return;
  }
  ctl_after_kkt(P, C);
}

// the control step after phase `op` and its reduction (C.rk, C.ra, C.rb);
// kept out of line (it runs on one thread; inlined into the driver it would
// add to the register pressure of every phase around it)
__device__ __attribute__((noinline)) void control(const SolveParams& P, Ctl& C, int op) {
  const Ctl& r = C;
  switch (op) {
    case OP_AX_START:
      C.exact = 1;
      C.op = OP_NSIDE;
      break;
    case OP_NSIDE:
      if (!P.qx || C.exact) C.S.qx_formed += 1;
      C.kc_exact = C.exact;
      C.exact = 0;
      if (C.retry) {  // x^k again for a repeated trial: only r_0 is needed
        C.retry = 0;
        C.rho = r.ra;
        ctl_start_cg(P, C, false);
        break;
      }
      C.kc = r.rk;
      C.rho = r.ra;
      C.tflag = r.rb;
      ctl_after_nside(P, C);
      break;
    case OP_DUAL_TRIAL: {
      // step limit of the trial (Sec. 4, adaptive step size: the PDLP rule
      // with the QP-specific term), ||dz||_w^2 / (2 |dy'A dx| + dx'Q dx) in
      // the primal-weight norm, +inf for a zero denominator; the trial is
      // accepted when eta <= eta_bar (or after 64 trials), and the step of the
      // next trial or iteration is min((1 - (t+1)^-0.3) eta_bar,
      // (1 + (t+1)^-0.6) eta) with t = k_total + 1 either way
      const double om = C.S.omega;
      const double num = om * C.rt[0] + C.rt[1] / om, den = 2.0 * fabs(C.rt[2]) + C.rt[3];
      const double eta_bar = den > 0.0 ? num / den : INFINITY;
      C.S.attempts += 1;
      const bool accept = C.S.eta <= eta_bar || C.S.attempts >= 64;
      const double t1 = (double)C.S.k_total + 2.0;
      const double ea = (1.0 - pow(t1, -0.3)) * eta_bar, eb = (1.0 + pow(t1, -0.6)) * C.S.eta;
      C.S.eta = ea < eb ? ea : eb;
      C.S.tau = C.S.eta / om;
      C.S.sigma = C.S.eta * om;
      if (accept) {
        C.S.attempts = 0;
        C.op = OP_COMMIT;
      } else {
        C.S.rejections += 1;
        C.op = OP_RETRY;
      }
      break;
    }
    case OP_RETRY:
      C.retry = 1;
      C.op = OP_NSIDE;
      break;
    case OP_ZERO:
      C.op = OP_AX_ZERO;
      break;
    case OP_AX_ZERO:
      C.S.cold_fallback = 1;
      C.exact = 1;
      C.op = OP_NSIDE;
      break;
    case OP_CERTIFY:
      C.kc = r.rk;
      if (C.kc.kkt > P.tol) C.S.mixed = 0;  // the certificate failed: finish in FP64
      ctl_after_kkt(P, C);
      break;
    case OP_EVAL:
      C.ka = r.rk;
      ctl_after_eval(P, C);
      break;
    case OP_RESTART: {
      const double dx = sqrt(r.ra), dy = sqrt(r.rb);
      if (P.theta > 0.0 && dx > 1e-10 && dy > 1e-10)
        C.S.omega = exp(P.theta * log(dy / dx) + (1.0 - P.theta) * log(C.S.omega));
      C.S.tau = C.S.eta / C.S.omega;
      C.S.sigma = C.S.eta * C.S.omega;
      C.S.K_anchor = C.Kc;
      C.S.K_prev = INFINITY;
      C.S.k = 0;
      C.S.eps = 0.0;
      C.S.restarts += 1;
      C.have_avg = 0;
      C.exact = 1;
      if (C.use_avg)
        C.op = OP_NSIDE;  // the point moved: redo the n-side pass there
      else
        ctl_limits(P, C);
      break;
    }
    case OP_LIMIT_AX:
      C.kc = r.rk;
      ctl_limit_after_ax(P, C);
      break;
    case OP_LIMIT_EVAL:
      C.ka = r.rk;
      C.have_avg = 1;
      ctl_limit_report(P, C);
      break;
    case OP_CG: {
      const int l = C.l;
      if (l > 0) C.steps = l;
      if (l >= P.max_cg) {  // the last allowed step only advanced x
        ctl_end_cg(P, C);
        break;
      }
      if (l == 0) {
        C.alpha = C.gamma / r.rb;
        C.beta = 0.0;
        C.l = 1;
        break;
      }
      const double gl = r.ra, dl = r.rb;
      if ((P.cg_rule == 0 && C.S.tau * sqrt(gl) <= C.S.eps) || !(gl > 0.0)) {
        ctl_end_cg(P, C);
        break;
      }
      C.beta = gl / C.gamma;
      C.alpha = gl / (dl - C.beta * gl / C.alpha);
      C.gamma = gl;
      C.l = l + 1;
      break;
    }
    case OP_CG_SPMV:
      C.alpha = C.rho / r.ra;
      C.op = OP_CG_UPDATE;
      break;
    case OP_CG_UPDATE: {
      const double rho_new = r.ra;
      C.steps = C.l;
      if (C.l == P.max_cg || (P.cg_rule == 0 && C.S.tau * sqrt(rho_new) <= C.S.eps) || !(rho_new > 0.0)) {
        ctl_end_cg(P, C);
        break;
      }
      C.beta = rho_new / C.rho;
      C.rho = rho_new;
      C.first = 0;
      C.cur ^= 1;
      C.l += 1;
      C.op = OP_CG_SPMV;
      break;
    }
    case OP_DUAL:
    case OP_COMMIT:
      C.S.k += 1;
      C.S.k_total += 1;
      C.budget -= 1;
      // a kept Q x is formed anew at every restart evaluation, so its
      // rounding drift never spans more than eval_period iterations
      C.exact = C.S.k % P.eval_period == 0;
      C.op = C.budget > 0 ? OP_NSIDE : OP_END;
      break;
    default:
      C.op = OP_END;
  }
}

// The primal step's CG run as one chain, for a workgroup whose CG rows form
// one tile, whose rows of Q and CG state are held in LDS, with FP32 products:
// the same product phase per step as phase_cgcg, one grid barrier per step,
// the same reduction and control step.  What differs is the order after each
// barrier: the gathers of the next step's product (the interleaved (r, u, s)
// rows of the tile's columns, which need none of the scalars being reduced)
// are issued together with the loads of the step's partials, so one memory
// round trip serves both, and the next product is formed from those
// registers once the control step has set alpha and beta.  Entered at a
// product step (C.l < max_cg) after its control step; returns after the
// control step that ends the chain (C.op then names the next phase, which the
// caller runs), with the barrier's epoch and ok = 0 if a barrier failed.
struct ChainEnd {
  uint64_t epoch;
  int ok;
};

__device__ __forceinline__ ChainEnd cg_chain(const SolveParams& P, Block B, GridSync gs, Ctl& C,
                                                       double* lds) {
  const WgPart& pt = P.w_cg;
  const int32_t* t = pt.tile(pt.t0);
  const int nz = t[3] - t[2];
  const int zoff = t[2] - pt.e0;  // first entry of the tile in the LDS block
  const float* lval = (const float*)pt.lval;
  double* const ob = P.cg_own;
  const int ro0 = pt.r0, no = pt.r1 - pt.r0;
  const double inv_tau = C.inv_tau;  // fixed within a primal step
  float4 q[kStageUnroll];
  auto gather = [&](const float4* v) {  // raw rows of the tile's columns (no wait)
    if (nz > 0) {
      int c[kStageUnroll];
#pragma unroll
      for (int u = 0; u < kStageUnroll; ++u) c[u] = lld(pt.lcol + zoff + min(u * kBlock + B.tid, nz - 1));
#pragma unroll
      for (int u = 0; u < kStageUnroll; ++u) q[u] = gld(v + c[u]);
    }
  };
  // the CG coefficients and counters, kept uniform in registers during the
  // chain (every workgroup runs this code on the same reduced values) and
  // written back before the control step that ends it
  int l = C.l, steps = C.steps;
  double alpha = C.alpha, beta = C.beta, gamma = C.gamma;
  const double tau = C.S.tau, eps = C.S.eps;
  gather((l == 0 ? 0 : (l & 1) ^ 1) ? P.v32_1 : P.v32_0);
  for (;;) {
    float4* v_new = (l & 1) ? P.v32_1 : P.v32_0;
    auto stage = [&](TileLds& L, int ra, int nr, int z0, int nzt) {
#pragma unroll
      for (int u = 0; u < kRowsPerThread; ++u) {
        const int i = u * kBlock + B.tid;
        if (i <= nr) L.rp[i] = lld(pt.lrp + ra + i - ro0) - z0;
      }
#pragma unroll
      for (int u = 0; u < kStageUnroll; ++u) {
        const int k = u * kBlock + B.tid;
        if (k < nzt) {
          const double rj = q[u].x, uj = q[u].y, sj = q[u].z;
          const double s1 = l == 1 ? uj : uj + beta * sj;
          const double g = l == 0 ? rj : rj - alpha * s1;
          L.prod[k] = (double)lld(lval + zoff + k) * g;
        }
      }
    };
    struct Row {
      double rp, xp;
    };
    auto pre = [&](int i) {  // step 0 starts from r_0 and x in device memory
      if (l == 0) return Row{gld(P.r + i), gld(P.x + i)};
      return Row{0.0, 0.0};
    };
    double s2[2] = {0.0, 0.0};  // gamma_l, delta_l
    auto epi = [&](int i, double qr, const Row& rw) {
      double* const o = ob + (i - ro0);
      double ri, s1 = 0.0;
      if (l == 0) {
        lst(o, rw.xp);
        ri = rw.rp;
      } else {
        const double xp = lld(o), pp = lld(o + no), rp = lld(o + 2 * no), up = lld(o + 3 * no),
                     sp = lld(o + 4 * no);
        s1 = l == 1 ? up : up + beta * sp;
        const double pi = l == 1 ? rp : rp + beta * pp;
        const double xi = xp + alpha * pi;
        lst(o + no, pi);
        lst(o, xi);
        gst(P.x32 + i, (float)xi);
        ri = rp - alpha * s1;
        lst(o + 4 * no, s1);
      }
      lst(o + 2 * no, ri);
      const double ui = qr + ri * inv_tau;
      lst(o + 3 * no, ui);
      gst(v_new + i, make_float4((float)ri, (float)ui, (float)s1, 0.0f));
      s2[0] += ri * ri;
      s2[1] += ri * ui;
    };
    tile_rows_impl(t, pt.group, stage, pre, epi);
    double dummy[1] = {0.0};
    block_reduce<2, 0>(s2, dummy, lds);
    if (B.tid == 0) {
      P.part[S_RR * B.nb + B.b] = s2[0];
      P.part[S_PQ * B.nb + B.b] = s2[1];
    }
    if (!gs.sync()) return ChainEnd{gs.epoch, 0};
    gather(v_new);  // the next step reads the copy this step wrote
    const int ss[2] = {S_RR, S_PQ};
    const int ms[1] = {0};
    double gd[2], m0[1];
    reduce_partials<2, 0>(P.part, B.nb, ss, ms, gd, m0, lds);
    // the control step of a CG phase (control(), OP_CG) while the chain goes on
    const double gl = uniform(gd[0]), dl = uniform(gd[1]);
    const bool stop = l > 0 && ((P.cg_rule == 0 && tau * sqrt(gl) <= eps) || !(gl > 0.0));
    const int l_next = l + 1;
    if (!stop && l_next < P.max_cg) {
      if (l == 0) {
        alpha = gamma / dl;
        beta = 0.0;
      } else {
        steps = l;
        beta = gl / gamma;
        alpha = gl / (dl - beta * gl / alpha);
        gamma = gl;
      }
      l = l_next;
      continue;
    }
    // the chain ends here: the control step proper decides from the state
    // before this reduction (the end of the primal step, or its last step)
    if (B.tid == 0) {
      C.l = l;
      C.steps = steps;
      C.alpha = alpha;
      C.beta = beta;
      C.gamma = gamma;
      C.ra = gd[0];
      C.rb = gd[1];
      control(P, C, OP_CG);
    }
    __syncthreads();
    return ChainEnd{gs.epoch, 1};
  }
}

// Runs at most `budget` iterations from the state C.S (set by thread 0 before
// the call, updated in place); returns false only if a grid barrier failed.
template <bool DENSE>
__device__ bool drive(const SolveParams& P, Block B, GridSync& gs, Ctl& C, double nb_inf, double nc_inf,
                      double* lds, double* svec, int64_t budget) {
  if (B.tid == 0) {
    C.budget = budget;
    C.have_avg = 0;
    C.retry = 0;
    C.exact = 1;
    C.kc_exact = 0;
    C.op = C.S.done || budget <= 0 ? OP_END : (C.S.K_anchor != C.S.K_anchor ? OP_AX_START : OP_NSIDE);
  }
  __syncthreads();
  bool ok = true;
  const WgPart& pc = P.w_cg;
  const bool chain_ok = !DENSE && P.cg_chain && P.cg_own != nullptr && pc.lcol != nullptr;
  for (;;) {
    const int op = C.op;
    if (op == OP_END) break;
    const int mixed = C.S.mixed;
    if (op == OP_CG && mixed && chain_ok && C.l < P.max_cg) {
      const ChainEnd e = cg_chain(P, B, gs, C, lds);
      gs.epoch = e.epoch;
      if (!(ok = e.ok != 0)) break;
      continue;
    }
    if (!DENSE && P.lr_d && (op == OP_NSIDE || op == OP_EVAL || op == OP_LIMIT_EVAL || op == OP_CG_SPMV)) {
      // low-rank Q: t = P' v first (one more grid barrier per product)
      if (op == OP_CG_SPMV) {
        const int cur = C.cur;
        if (mixed)
          phase_lr_t(P, B, P.Lt.val32, GatherDir2{P.rp32, C.beta, C.first}, lds);
        else
          phase_lr_t(P, B, P.Lt.val, GatherDir<double>{P.r, cur ? P.p0 : P.p1, C.beta, C.first}, lds);
      } else {
        phase_lr_t(P, B, P.Lt.val, GatherVec<double>{op == OP_NSIDE ? P.x : P.xa}, lds);
      }
      if (!(ok = gs.sync())) break;
    }
    switch (op) {
      case OP_AX_START:
      case OP_AX_ZERO:
      case OP_CERTIFY:
      case OP_LIMIT_AX:
        phase_ax(P, B, lds);
        break;
      case OP_NSIDE:
        // r_0 in FP32 goes where the next product gathers it: the interleaved
        // (r, u, s) rows of the single-reduction CG, or the plain copy
        if (P.v32_0)
          phase_nside<DENSE>(P, P.w_n1, B, P.x, P.y, P.r, mixed ? (float*)P.v32_0 : nullptr, 4, 0, lds, svec);
        else
          phase_nside<DENSE>(P, P.w_n1, B, P.x, P.y, P.r, mixed ? (float*)P.rp32 : nullptr, 2, 0, lds, svec,
                             P.qx ? (C.exact ? QX_FORM : QX_KEPT) : QX_INTO_Q);
        if (B.tid == 0) {
          double f = 0.0;
          if (B.b == 0 && P.time_limit_ticks && wall_clock64() - C.S.t_start > P.time_limit_ticks) f = 1.0;
          P.part[S_FLAG * B.nb + B.b] = f;
        }
        break;
      case OP_ZERO:
        phase_zero_point(P, B);
        break;
      case OP_EVAL:
      case OP_LIMIT_EVAL:
        phase_eval_avg<DENSE>(P, B, lds, svec);
        break;
      case OP_RESTART:
        phase_restart(P, B, C.use_avg, mixed, lds);
        break;
      case OP_CG:
        if (mixed && P.cg_own)
          phase_cgcg<float, float, true>(P, B, P.Q.val32, C.l, C.alpha, C.beta, C.inv_tau, C.l < P.max_cg, 1, lds);
        else if (mixed)
          phase_cgcg<float, float, false>(P, B, P.Q.val32, C.l, C.alpha, C.beta, C.inv_tau, C.l < P.max_cg, 1, lds);
        else if (P.cg_own)
          phase_cgcg<double, double, true>(P, B, P.Q.val, C.l, C.alpha, C.beta, C.inv_tau, C.l < P.max_cg, 0, lds);
        else
          phase_cgcg<double, double, false>(P, B, P.Q.val, C.l, C.alpha, C.beta, C.inv_tau, C.l < P.max_cg, 0, lds);
        break;
      case OP_CG_SPMV: {
        const int cur = C.cur;
        double* pc = cur ? P.p1 : P.p0;
        const double* pp = cur ? P.p0 : P.p1;
        if (mixed)
          phase_cg_spmv<DENSE>(P, B, P.Q.val32, GatherDir2{P.rp32, C.beta, C.first}, pp, pc, C.beta, C.first,
                               C.inv_tau, lds, svec);
        else
          phase_cg_spmv<DENSE>(P, B, P.Q.val, GatherDir<double>{P.r, pp, C.beta, C.first}, pp, pc, C.beta, C.first,
                               C.inv_tau, lds, svec);
        break;
      }
      case OP_CG_UPDATE:
        phase_cg_update(P, B, C.cur ? P.p1 : P.p0, C.alpha, mixed, C.inv_tau, lds);
        break;
      case OP_DUAL:
        if (mixed)
          phase_dual(P, B, P.A.val32, (const float*)P.x32, C.S.sigma, C.w, C.xlds ? P.cg_own : nullptr, lds);
        else
          phase_dual(P, B, P.A.val, (const double*)P.x, C.S.sigma, C.w, C.xlds ? P.cg_own : nullptr, lds);
        break;
      case OP_DUAL_TRIAL:
        // with FP32 values of A, x is gathered in FP64: A x' and the A x^k of
        // the previous trial then share the rounding of A, and dy.(A x' - A x^k)
        // in the step limit keeps its accuracy as the steps shrink (the rounding
        // of x to FP32 would not cancel)
        if (mixed)
          phase_dual_trial<DENSE>(P, B, P.A.val32, (const double*)P.x, C.S.sigma, lds, svec);
        else
          phase_dual_trial<DENSE>(P, B, P.A.val, (const double*)P.x, C.S.sigma, lds, svec);
        break;
      case OP_COMMIT:
        phase_commit(P, B, C.w);
        break;
      case OP_RETRY:
        phase_retry(P, B);
        break;
      case OP_COPY_AVG:
        phase_copy_point(P, B, P.xa, P.ya);
        break;
      case OP_COPY_ANCHOR:
        phase_copy_point(P, B, P.x_anc, P.y_anc);
        break;
    }
    if (op == OP_COPY_AVG || op == OP_COPY_ANCHOR) break;  // the solve ends with this copy
    if (!(ok = gs.sync())) break;
    double a = 0.0, b = 0.0;
    switch (op) {
      case OP_NSIDE:
        reduce_kkt(P, B, 0, nb_inf, nc_inf, &C.rk, &C.ra, &C.rb, lds);
        break;
      case OP_CERTIFY:
      case OP_LIMIT_AX:
        reduce_kkt(P, B, 0, nb_inf, nc_inf, &C.rk, nullptr, nullptr, lds);
        break;
      case OP_EVAL:
      case OP_LIMIT_EVAL:
        reduce_kkt(P, B, S_AVG0, nb_inf, nc_inf, &C.rk, nullptr, nullptr, lds);
        break;
      case OP_RESTART: {
        const int ss[2] = {S_DX, S_DY};
        const int ms[1] = {0};
        double s2[2], m0[1];
        reduce_partials<2, 0>(P.part, B.nb, ss, ms, s2, m0, lds);
        a = s2[0];
        b = s2[1];
        break;
      }
      case OP_CG:
        if (C.l < P.max_cg) {
          const int ss[2] = {S_RR, S_PQ};
          const int ms[1] = {0};
          double gd[2], m0[1];
          reduce_partials<2, 0>(P.part, B.nb, ss, ms, gd, m0, lds);
          a = gd[0];
          b = gd[1];
        }
        break;
      case OP_CG_SPMV:
        a = reduce_one(P, B, S_PQ, lds);
        break;
      case OP_CG_UPDATE:
        a = reduce_one(P, B, S_RR, lds);
        break;
      case OP_DUAL_TRIAL: {
        const int ss[4] = {S_DX2, S_DY2, S_DYADX, S_DXQDX};
        const int ms[1] = {0};
        double t4[4], m0[1];
        reduce_partials<4, 0>(P.part, B.nb, ss, ms, t4, m0, lds);
        if (B.tid == 0)
          for (int k = 0; k < 4; ++k) C.rt[k] = t4[k];
        break;
      }
      default:
        break;
    }
    if (B.tid == 0) {
      if (op != OP_NSIDE) {  // (the n-side reduction wrote its own scalars)
        C.ra = a;
        C.rb = b;
      }
      control(P, C, op);
    }
    __syncthreads();
  }
  return ok;
}

// The workgroup's share of a row partition, for its LDS copy of the
// parameter block.
__device__ void fill_wg_part(WgPart& w, const Part& p, int b) {
  const int t0 = p.tile_ptr[b], t1 = p.tile_ptr[b + 1];
  if (threadIdx.x == 0) {
    w.r0 = p.bounds[b];
    w.r1 = p.bounds[b + 1];
    w.t0 = t0;
    w.t1 = t1;
    w.l0 = p.long_ptr[b];
    w.l1 = p.long_ptr[b + 1];
    w.group = p.group;
    w.tiles = p.tiles;
    w.long_rows = p.long_rows;
    w.e0 = 0;
    w.lrp = nullptr;
    w.lcol = nullptr;
    w.lval = nullptr;
  }
  const int nt = t1 - t0 < kCacheTiles ? t1 - t0 : kCacheTiles;
  for (int k = threadIdx.x; k < 6 * nt; k += kBlock) w.tl[k] = p.tiles[6 * t0 + k];
}

// Copy the parameter block into LDS and cache the workgroup's share of the
// row partitions there: the phases then read pointers, sizes and tile
// descriptors at LDS latency instead of through the L2 that every grid
// barrier invalidates.
__device__ void load_params(SolveParams& Ps, const SolveParams* Pg, int b) {
  static_assert(sizeof(SolveParams) % 8 == 0, "parameter block copied in 8-byte words");
  const uint64_t* src = (const uint64_t*)Pg;
  uint64_t* dst = (uint64_t*)&Ps;
  for (int k = threadIdx.x; k < (int)(sizeof(SolveParams) / 8); k += kBlock) dst[k] = src[k];
  __syncthreads();
  fill_wg_part(Ps.w_n1, Ps.pn1, b);
  fill_wg_part(Ps.w_cg, Ps.pcg, b);
  fill_wg_part(Ps.w_m, Ps.pm, b);
  if (Ps.lr_d) fill_wg_part(Ps.w_lr, Ps.plr, b);
  __syncthreads();
}

// ||A||_2 by power iteration on A'A (the step-size rule of Thm 2 needs it;
// the paper does not say how it is obtained): start from
// v_j = 0.5 + ((j * 40503) mod 1024) / 1024, normalised; each step
// u = A v, w = A'u, lambda = ||w||, v = w / lambda; ||A|| ~ sqrt(lambda).
// v, w (n) and u (m) are work vectors; pn partitions the rows of A', pm
// those of A.  Returns false if a grid barrier failed.
__device__ bool power_norm(const DevMat& A, const DevMat& At, double* v, double* w, double* u, double* part,
                           const Part& pn, const Part& pm, int iters, Block B, GridSync& gs, double* lds,
                           double* out) {
  const int n0 = pn.bounds[B.b], n1 = pn.bounds[B.b + 1];
  double s[1] = {0.0}, dummy[1] = {0.0};
  for (int j = n0 + B.tid; j < n1; j += kBlock) {
    const double vj = 0.5 + (double)(((uint64_t)j * 40503ull) % 1024ull) / 1024.0;
    w[j] = vj;
    s[0] += vj * vj;
  }
  block_reduce<1, 0>(s, dummy, lds);
  if (B.tid == 0) part[S_PW * B.nb + B.b] = s[0];
  if (!gs.sync()) return false;
  const int ss[1] = {S_PW};
  const int ms[1] = {0};
  double tot[1], m0[1];
  reduce_partials<1, 0>(part, B.nb, ss, ms, tot, m0, lds);
  double scale = 1.0 / sqrt(tot[0]);
  double lam = 0.0;
  for (int it = 0; it < iters; ++it) {
    for (int j = n0 + B.tid; j < n1; j += kBlock) v[j] = w[j] * scale;
    if (!gs.sync()) return false;
    {  // u = A v
      GatherVec<double> gv{v};
      for (int t = pm.tile_ptr[B.b]; t < pm.tile_ptr[B.b + 1]; ++t)
        tile_rows(A.rowptr, A.col, A.val, pm.tiles + 6 * t, pm.group, gv, [&](int i, double su) { u[i] = su; });
      for (int t = pm.long_ptr[B.b]; t < pm.long_ptr[B.b + 1]; ++t) {
        const int i = pm.long_rows[t];
        double vv[1] = {row_partial(A.col, A.val, A.rowptr[i], A.rowptr[i + 1], B.tid, kBlock, gv)};
        block_reduce<1, 0>(vv, dummy, lds);
        if (B.tid == 0) u[i] = vv[0];
      }
    }
    if (!gs.sync()) return false;
    {  // w = A'u, partial ||w||^2
      GatherVec<double> gu{u};
      double sw[1] = {0.0};
      for (int t = pn.tile_ptr[B.b]; t < pn.tile_ptr[B.b + 1]; ++t)
        tile_rows(At.rowptr, At.col, At.val, pn.tiles + 6 * t, pn.group, gu, [&](int i, double st) {
          w[i] = st;
          sw[0] += st * st;
        });
      for (int t = pn.long_ptr[B.b]; t < pn.long_ptr[B.b + 1]; ++t) {
        const int i = pn.long_rows[t];
        double vv[1] = {row_partial(At.col, At.val, At.rowptr[i], At.rowptr[i + 1], B.tid, kBlock, gu)};
        block_reduce<1, 0>(vv, dummy, lds);
        if (B.tid == 0) {
          w[i] = vv[0];
          sw[0] += vv[0] * vv[0];
        }
      }
      block_reduce<1, 0>(sw, dummy, lds);
      if (B.tid == 0) part[S_PW * B.nb + B.b] = sw[0];
    }
    if (!gs.sync()) return false;
    reduce_partials<1, 0>(part, B.nb, ss, ms, tot, m0, lds);
    lam = sqrt(tot[0]);
    if (!(lam > 0.0)) break;
    scale = 1.0 / lam;
  }
  *out = sqrt(lam);
  return true;
}

// ------------------------------------------------------- cooperative solve

// Copy the workgroup's rows of M (row pointers, columns, values of vbytes)
// into its resident block at base and record the block in w.
__device__ __forceinline__ void place_resident(WgPart& w, const DevMat& M, char* base, int vbytes) {
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

// The cooperative solve of one QP (the body of the solve kernels of both
// workgroup sizes): parameter block and partition share into LDS, the rows
// planned resident copied there, then the driver; the state goes back to
// device memory at the end (or a barrier failure is flagged).
__device__ __forceinline__ void solve_body(const SolveParams* __restrict__ Pg) {
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

// -------------------------------------------------------------- batched solve

// One workgroup per QP: workgroup g solves instance order[g] (the host sorts
// instances by decreasing work, so the dispatcher hands out the largest
// first).  Each workgroup runs the same loop as the cooperative kernel with
// nb = 1 (a grid barrier degenerates to a workgroup barrier), on its own slice
// of the packed matrices and vectors; dense Q blocks use the streaming dense
// product.  ||A|| comes from the same power iteration, per instance.
__device__ __forceinline__ void batch_solve(const BatchParams& BP) {
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

// ||A||_2 by the power iteration on A'A, every workgroup taking its rows of
// A' and A (the launch of the single-QP path before its first solve)
__device__ __forceinline__ void power_body(const PowerParams& P) {
  __shared__ double lds[kWaves * 8];
  Block B{(int)blockIdx.x, (int)gridDim.x, (int)threadIdx.x};
  GridSync gs{P.bar, (uint32_t)gridDim.x, 0};
  if (!gs.init()) return;  // (the host finds the abort word raised)
  double nrm = 0.0;
  if (power_norm(P.A, P.At, P.v, P.w, P.u, P.part, P.pn, P.pm, P.iters, B, gs, lds, &nrm) && B.b == 0 &&
      B.tid == 0)
    P.out[0] = nrm;
}

}  // namespace
}  // namespace pdhcg
