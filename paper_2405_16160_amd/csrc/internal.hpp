// Internal definitions shared by the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdhcg {

// Threads per workgroup.  The cooperative single-QP kernels run 512 (one
// workgroup per CU); the batched kernel, one workgroup per QP, runs 256 by
// default so that two instances share a CU at the same register budget (two
// waves per SIMD), or 512 (one instance per CU) when its autotuner finds that
// faster.  The solver's device code is compiled once per size: a translation
// unit that defines PDHCG_BLOCK_SIZE gets that size, the others 512.
constexpr int kSolveBlock = 512;
constexpr int kBatchBlock = 256;
#ifdef PDHCG_BLOCK_SIZE
constexpr int kBlock = PDHCG_BLOCK_SIZE;
#else
constexpr int kBlock = kSolveBlock;
#endif
constexpr int kBarWords = 2048;   // grid-barrier words (uint64) per handle, zeroed before each launch
constexpr int kBarAbortWord = 64; // the barrier word raised when a wait timed out
constexpr int kWave = 64;         // CDNA wavefront
constexpr int kWaves = kBlock / kWave;
constexpr int kLongRow = 1024;    // rows longer than this are reduced by the whole workgroup

// Device CSR with 32-bit indices; val32 is an FP32 copy of val (or null).
// dense = 1 marks a square matrix stored as nrows*ncols row-major values
// (rowptr and col unused); only the one-workgroup-per-QP kernel takes it.
struct DevMat {
  int32_t nrows, ncols;
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  const float* val32;
  int32_t dense;     // 0 CSR; 1 dense n x n rows; 2 Q = F F' + diag(d) from its factor (batch only)
  int32_t rank;      // k of the factor when dense = 2 (0 otherwise)
};

constexpr int kDenseTile = 2048;  // doubles of the LDS tile that stages the vector of a dense product
constexpr int kDenseRows = 4;     // rows per thread in one pass of a dense product

// Static partition of a row space over the workgroups of a solve kernel.
// Workgroup w owns rows [bounds[w], bounds[w+1]); rows of that range longer
// than kLongRow are listed in long_rows[long_ptr[w] .. long_ptr[w+1]) and are
// reduced cooperatively by the whole workgroup; the others are reduced by
// groups of `group` lanes (a power of two <= 64).
//
// The other rows of a workgroup's range are cut into tiles of at most
// kTileNnz entries and kTileRows rows: tiles[6*t .. 6*t+5] = first row, end
// row, entry range in the first matrix, entry range in the second matrix (for
// the stacked [Q | A'] pass; zero otherwise); workgroup w owns tiles
// tile_ptr[w] .. tile_ptr[w+1]-1.  A tile's products are staged in LDS with
// all loads in flight at once and then reduced row by row from LDS.
struct Part {
  const int32_t* bounds;
  const int32_t* long_ptr;
  const int32_t* long_rows;
  const int32_t* tile_ptr;
  const int32_t* tiles;
  int32_t group;
};

// bytes of a workgroup's resident block: row pointers, columns, values (each 16-byte aligned)
__host__ __device__ inline int64_t align16(int64_t b) { return (b + 15) & ~(int64_t)15; }
__host__ __device__ inline int64_t res_block_bytes(int64_t nrows, int64_t ne, int vbytes) {
  return align16(4 * (nrows + 1)) + align16(4 * ne) + align16((int64_t)vbytes * ne);
}

// staged products (FP64 in LDS) and rows per tile of a workgroup of `block`
// threads: 8 entries and 2 rows per thread
constexpr int tile_nnz_for(int block) { return 8 * block; }
constexpr int tile_rows_for(int block) { return 2 * block; }
constexpr int kTileNnz = tile_nnz_for(kBlock);
constexpr int kTileRows = tile_rows_for(kBlock);

// One workgroup's share of a Part, cached in LDS when a solve kernel starts:
// owned rows [r0, r1), tiles t0 .. t1-1 (the first kCacheTiles of them copied
// into tl), long rows long_rows[l0 .. l1-1].
constexpr int kCacheTiles = 16;
struct WgPart {
  int32_t r0, r1, t0, t1, l0, l1, group;
  int32_t e0;               // first entry of row r0 (resident block)
  const int32_t* tiles;
  const int32_t* long_rows;
  // the workgroup's rows of the matrix held in LDS for the whole launch (null
  // when not held): lrp[j] = rowptr[r0 + j], lcol / lval = entries from e0
  const int32_t* lrp;
  const int32_t* lcol;
  const void* lval;
  int32_t tl[6 * kCacheTiles];
  __device__ __forceinline__ const int32_t* tile(int t) const {
    return t - t0 < kCacheTiles ? tl + 6 * (t - t0) : tiles + 6 * t;
  }
};

// Partial-result slots.  Every workgroup writes one value per slot; after a
// grid barrier every workgroup reduces all of them in the same fixed order,
// so every workgroup holds bit-identical scalars and takes the same decisions.
enum Slot {
  // n-side pass at the current point: g = Qx + A'y + c
  S_GG = 0,      // sum g^2                (= rho_0 of CG: r_0 = -g)
  S_MG,          // max |g|
  S_MQX,         // max |Qx|
  S_MATY,        // max |A'y|
  S_XQX,         // sum x.Qx
  S_CX,          // sum c.x
  // m-side pass at the current point: u = Ax
  S_MVIOL,       // max (u - b)^+
  S_MAX,         // max |u|
  S_BY,          // sum b.y
  // the same nine quantities at the running average
  S_AVG0,
  S_AVG_END = S_AVG0 + 9,
  // CG and restart
  S_PQ = S_AVG_END,  // sum p.q
  S_RR,          // sum r.r
  S_DX,          // sum (x_c - x_anchor)^2
  S_DY,          // sum (y_c - y_anchor)^2
  S_FLAG,        // max of a per-workgroup flag (time limit)
  S_PW,          // power iteration: sum w^2
  // adaptive step size: m-side partials of a trial point (max (u - b)^+,
  // max |u|, sum b.y), and the pieces of its step limit: sum dx^2, sum dy^2,
  // sum dy.(A dx), sum dx.(Q dx) for dx = x' - x, dy = y' - y
  S_TVIOL,
  S_TMAX,
  S_TBY,
  S_DX2,
  S_DY2,
  S_DYADX,
  S_DXQDX,
  NSLOT
};

// Scalar state of a solve; every workgroup keeps an identical copy in
// registers, workgroup 0 stores it here when a launch ends.
struct SolverState {
  int64_t k;            // iterations in the current epoch
  int64_t k_total;      // iterations in all epochs
  int64_t cg_total;     // CG steps
  int64_t restarts;
  int64_t evals;        // restart evaluations
  double eps;           // CG tolerance epsilon_k of the current epoch
  double K_anchor;      // relKKT of the epoch's starting point (NaN: not yet known)
  double K_prev;        // candidate relKKT at the previous evaluation of this epoch
  double omega, tau, sigma;
  double eta;           // eta_factor / ||A||_2
  int32_t done;         // 1 once a final status is set
  int32_t status;
  int32_t returned_average;
  int32_t mixed;        // 1 while FP32 products are in use
  int32_t start_checked;  // the start point's relKKT has been compared with (0, 0)'s
  int32_t cold_fallback;  // the start point was replaced by (0, 0)
  double r_p, r_d, r_g, kkt, pobj, dobj;  // of the returned point
  double norm_A;        // ||A||_2 estimate (batched solves)
  uint64_t t_start;     // wall_clock64() at the start of the solve
  int64_t rejections;   // rejected trial steps (adaptive step size)
  int32_t attempts;     // trials of the current iteration (adaptive step size)
  int32_t pad_;
  int64_t qx_formed;    // n-side passes at the current point that formed Q x with a product
};

struct SolveParams {
  DevMat Q, A, At;
  const double* b;
  const double* c;
  int32_t n, m;
  // iterate state (FP64)
  double *x, *y, *xa, *ya, *ax, *ax_avg, *x_anc, *y_anc;
  // CG work vectors (FP64)
  double *r, *p0, *p1, *q;
  // one-reduction CG (cooperative kernel): second r buffer, u = (Q + I/tau) r
  // and s = (Q + I/tau) p, double-buffered (null in the batched kernel)
  double *r_alt, *u0, *u1, *s0, *s1;
  // FP32 copies used by the mixed-precision products: x32; rp32 holds (r, p)
  // of the textbook CG per row, the residual and the direction of the last
  // update, so that a product's gather of p = r + beta p_prev reads one
  // 8-byte record (one cache line) per entry; v32_0 / v32_1 hold (r, u, s) of
  // the one-reduction CG interleaved per row (null in the batched kernel)
  float* x32;
  float2* rp32;
  float4 *v32_0, *v32_1;
  double* lr_t;  // k-vector F' v of a factored dense Q (batch only)
  double* part;         // [NSLOT][nb]
  uint64_t* bar;        // grid barrier words (zeroed before each launch)
  SolverState* st;
  Part pn1, pcg, pm, pt;  // n-side pass, CG (rows of Q), A rows, A' rows
  // the executing workgroup's share of pn1, pcg, pm (filled in its LDS copy of
  // this block; unused in the copy in device memory)
  WgPart w_n1, w_cg, w_m;
  // Q = P P' + diag(d) given by a sparse P (n x k) on a single-QP handle
  // (lr_d null otherwise): the Q above is then P itself, Lt its transpose
  // (k x n) with the row partition plr (w_lr: the workgroup's share), and
  // every product with Q first forms t = P' v into lr_pt (FP64) and lr_pt32
  // (its FP32 copy), then (Q v)_i = (P t)_i + d_i v_i
  DevMat Lt;
  Part plr;
  WgPart w_lr;
  const double* lr_d;
  double* lr_pt;
  float* lr_pt32;
  // LDS residency of Q (CG product rows) and A (dual product rows) in the
  // cooperative kernel: flags, value bytes (4: FP32 copies, 8: FP64), byte
  // offset of the A block in dynamic LDS
  int32_t res_cg, res_m, res_vbytes, res_m_off;
  // the single-reduction CG's state on the workgroup's CG rows (x, p, r, u,
  // s in FP64, five arrays of r1 - r0 values) held in LDS across the steps of
  // a primal step: flag, byte offset in dynamic LDS, and the block of the
  // executing workgroup (set in its LDS copy of this block; null otherwise)
  int32_t own_cg, own_off;
  double* cg_own;
  // FP32 products, Q rows and CG state in LDS and one CG tile per workgroup in
  // every workgroup: the CG steps run chained (cg_chain)
  int32_t cg_chain;
  double nb_inf, nc_inf;  // ||b||_inf, ||c||_inf of the caller's problem (enter every relKKT)
  // diagonal preconditioning: the data above are D2 Q D2, D1 A D2, D1 b, D2 c
  // and the iterates (x~, y~) stand for x = D2 x~, y = D1 y~ of the caller's
  // problem; every relKKT is taken there, so the residual maxima of row j
  // (i) are divided by dn[j] = D2_j (dm[i] = D1_i).  Null when not scaled.
  const double* dn;
  const double* dm;
  double kkt_zero;        // relKKT(0, 0) when the warm-start fallback applies, else 0
  // start point of a batched solve (null: zero)
  const double* x0;
  const double* y0;
  // settings
  double tol, eps_factor, beta_suf, beta_nec, beta_art, theta;
  int64_t max_iters;
  int64_t iters_this_launch;   // bound on iterations per launch
  uint64_t time_limit_ticks;   // 0 = none; wall_clock64() ticks
  int32_t max_cg, cg_rule, restart_to, eval_period;
  int32_t mixed_allowed;
  // adaptive step size (step_rule = 1): the point x^k of the iteration (saved
  // by the n-side pass), and the trial dual point and its A x' (m)
  int32_t step_rule;
  // Q x of the current point kept by linearity (a dense or factored Q in the
  // batch with the constant step rule; null otherwise): the n-side pass then
  // forms Q x with a product only every eval_period iterations, after a
  // restart and before a termination or a limit is reported, and reads the
  // kept vector in between
  double* qx;
  double* x_prev;
  double* y_trial;
  double* ax_trial;
};

struct PowerParams {
  DevMat A, At;
  double* v;     // n
  double* w;     // n
  double* u;     // m
  double* part;
  uint64_t* bar;
  double* out;   // [0] = ||A|| estimate
  Part pn, pm;
  int32_t iters;
};

// Batched solve: params[i] describes QP i (pointers into the packed device
// arrays, its row partitions for one workgroup, its x0/y0); workgroup g
// solves QP order[g].  Parameter blocks are written by the host before the
// launch and only read by the kernel.
struct BatchParams {
  const SolveParams* params;
  const int32_t* order;
  SolverState* st;           // [count] results
  uint64_t* t0;              // wall clock at the start of the batch
  double pw_init, eta_factor;
  int32_t power_iters;
  int32_t mixed;
  // per instance: bit 0 = x0 given, bit 1 = y0 given (the parameter blocks
  // always point at the packed start buffers; without the bit the start is 0)
  const uint8_t* given;
  int32_t warm_fallback;  // compare a given start with (0, 0) (params' kkt_zero)
};

// records the message returned by pdhcg_last_error() and returns code
int set_error(int code, const char* msg);

}  // namespace pdhcg
#include "../../include/pdhcg.h"
namespace pdhcg {
// pdhcg_solve_batch with every device buffer carved from the given device
// region (region_bytes long) instead of allocated: INVALID_ARGUMENT when the
// batch does not fit
int solve_batch_in_region(int32_t count, const pdhcg_csr* Qs, const pdhcg_csr* As, const double* const* bs,
                          const double* const* cs, const double* const* x0s, const double* const* y0s,
                          double* const* x_outs, double* const* y_outs, pdhcg_result* rs, const pdhcg_settings* s,
                          void* hip_stream, char* region, size_t region_bytes);

// the batched kernel with 256 (batch_kernels.hip) or 512 threads per
// workgroup (batch_kernels_512.hip); the clock kernel stamps the batch's start
hipError_t launch_batch_clock(uint64_t* t0, hipStream_t s);
hipError_t launch_batch_256(const BatchParams& p, int count, hipStream_t s);
hipError_t launch_batch_512(const BatchParams& p, int count, hipStream_t s);
// the cooperative kernels at `threads` per workgroup (512: solve_kernels.hip;
// 256: solve_kernels_256.hip, whose kernels solve_kernel_256() and
// power_kernel_256() return)
hipError_t launch_solve(int threads, const SolveParams* p_dev, int nb, int dyn_lds, hipStream_t s);
const void* solve_kernel_256();
const void* power_kernel_256();
// static LDS bytes of the solve kernel, and the co-resident workgroups per CU
// it reaches with dyn_lds bytes of dynamic LDS
hipError_t solve_kernel_lds(int threads, int* static_bytes);
hipError_t solve_occupancy_dyn(int threads, int dyn_lds, int* per_cu);
hipError_t launch_power(int threads, const PowerParams& p, int nb, hipStream_t s);
hipError_t launch_init_point(const SolveParams* p_dev, int64_t n, int64_t m, hipStream_t s);
// standalone product y = M x over host-cut tiles (spmv_kernels.hip)
hipError_t launch_spmv_stream(const int32_t* rowptr, const int32_t* col, const double* val, const float* val32,
                              int precision, const double* x, const float* x32, double* y, const int32_t* tiles,
                              int ntiles, hipStream_t s);
int spmv_stream_tile_nnz();
int spmv_stream_tile_rows();
hipError_t launch_to_f32(const double* in, float* out, int64_t n, hipStream_t s);
// diagonal preconditioning (precond_kernels.hip): ruiz_iters Ruiz steps and an
// optional Pock-Chambolle step on [[Q, A'], [A, 0]], applied to the FP64 values
// of Q, A and T = A' in place (CSR, row pointers relative to the col/val
// pointers); f is scratch of n + m doubles; d2 (n) and d1 (m), set to 1 by
// the caller, accumulate D2 and D1; nnzq, nnza are the entry counts of Q and
// A (they size the lane groups per row)
hipError_t launch_precondition(const DevMat& Q, const DevMat& A, const DevMat& T, int64_t nnzq, int64_t nnza,
                               int ruiz_iters, int pock_chambolle, double* f, double* d2, double* d1, hipStream_t s);
// One instance of a batched preconditioning (launch_batch_precondition): its
// blocks in the packed batch arrays, scaled in place; Q is CSR (qkind 0), a
// dense n x n block (1) or the factor block [F (n x k) | F' (k x n) | d (n)]
// of Q = F F' + diag(d) (2); d2 (n) and d1 (m) hold ones on entry and receive
// D2, D1; f is scratch of n + m doubles; gk, gq, ga, gt are the lanes per row
// of the rows of K and of Q, A, A' (powers of two up to 64).
struct PrecInst {
  int32_t n, m, qkind, k;
  const int32_t* qrp;
  const int32_t* qcol;
  double* qval;
  const int32_t* arp;
  const int32_t* acol;
  double* aval;
  const int32_t* trp;
  const int32_t* tcol;
  double* tval;
  double* d2;
  double* d1;
  double* f;
  int32_t gk, gq, ga, gt;
};
// one workgroup per instance, every step in one launch
hipError_t launch_batch_precondition(const PrecInst* insts, int count, int ruiz_iters, int pock_chambolle,
                                     hipStream_t s);
// lanes per row the preconditioning kernels give rows of mean length nnz / nrows
int precond_lanes(int64_t nnz, int64_t nrows);
// out = x .* scale (op 0) or x ./ scale (op 1), n entries; out may be x
hipError_t launch_diag(const double* x, const double* scale, int64_t n, int op, double* out, hipStream_t s);
// workgroups per CU that the persistent kernels can keep resident (the
// smaller of the solve and power kernels)
hipError_t solve_occupancy(int threads, int* per_cu);

}  // namespace pdhcg
