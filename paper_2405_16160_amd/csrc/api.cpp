// Host side of the C ABI in include/pdhcg.h: input validation, A' build,
// row-partition planning, device uploads, and the solve driver that launches
// the persistent kernel and reads back its scalar state.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <limits>
#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/pdhcg.h"
#include "internal.hpp"

using namespace pdhcg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

int pdhcg::set_error(int code, const char* msg) { return fail(code, msg); }

namespace {

#define HIPX(call)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return fail(PDHCG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// relKKT at x = 0, y = 0: Ax = Qx = A'y = 0, so r_primal = max((-b)^+) /
// (1 + ||b||_inf), r_dual = ||c||_inf / (1 + ||c||_inf), r_gap = 0
double kkt_at_zero(const double* b, int64_t m, const double* c, int64_t n) {
  double viol = 0.0, bi = 0.0, ci = 0.0;
  for (int64_t i = 0; i < m; ++i) {
    viol = std::max(viol, -b[i]);
    bi = std::max(bi, fabs(b[i]));
  }
  for (int64_t j = 0; j < n; ++j) ci = std::max(ci, fabs(c[j]));
  return std::max(viol / (1.0 + bi), ci / (1.0 + ci));
}

double max_abs_nan(const double* v, int64_t n) {
  double m = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double a = fabs(v[i]);
    if (a != a) return a;
    if (a > m) m = a;
  }
  return m;
}

struct HostCsr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rowptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

// CSR structure checks on host arrays: rowptr[0] = 0, rowptr[nrows] = nnz,
// monotone rowptr, columns in range and strictly increasing within a row.
int check_structure(const int64_t* rowptr, const int32_t* col, int64_t nrows, int64_t ncols, int64_t nnz,
                    const std::string& name) {
  if (rowptr[0] != 0 || rowptr[nrows] != nnz)
    return fail(PDHCG_ERR_INVALID_ARGUMENT, name + ": rowptr[0] != 0 or rowptr[nrows] != nnz");
  // every row pointer is checked before any column is read, so that a bad
  // pointer cannot send the column scan past the end of col
  for (int64_t i = 0; i < nrows; ++i)
    if (rowptr[i + 1] < rowptr[i] || rowptr[i + 1] > nnz)
      return fail(PDHCG_ERR_INVALID_ARGUMENT,
                  name + ": rowptr not monotone or beyond nnz at row " + std::to_string(i));
  for (int64_t i = 0; i < nrows; ++i) {
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      if (col[k] < 0 || col[k] >= ncols)
        return fail(PDHCG_ERR_INVALID_ARGUMENT, name + ": column out of range in row " + std::to_string(i));
      if (k > rowptr[i] && col[k] <= col[k - 1])
        return fail(PDHCG_ERR_INVALID_ARGUMENT, name + ": columns not strictly increasing in row " + std::to_string(i));
    }
  }
  return 0;
}

int fetch_csr(const pdhcg_csr* M, HostCsr& H, const char* name) {
  if (!M) return fail(PDHCG_ERR_INVALID_ARGUMENT, std::string(name) + ": null matrix");
  if (M->nrows < 0 || M->ncols < 0 || M->nnz < 0)
    return fail(PDHCG_ERR_INVALID_ARGUMENT, std::string(name) + ": negative size");
  if (M->nrows >= (1ll << 31) - 1 || M->ncols >= (1ll << 31) - 1 || M->nnz >= (1ll << 31) - 1)
    return fail(PDHCG_ERR_INVALID_ARGUMENT, std::string(name) + ": sizes beyond 32-bit indexing");
  H.nrows = M->nrows;
  H.ncols = M->ncols;
  H.rowptr.resize(M->nrows + 1);
  H.col.resize(M->nnz);
  H.val.resize(M->nnz);
  if (!M->rowptr || (M->nnz > 0 && (!M->col || !M->val)))
    return fail(PDHCG_ERR_INVALID_ARGUMENT, std::string(name) + ": null array");
  hipMemcpyKind kind = M->on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  HIPX(hipMemcpy(H.rowptr.data(), M->rowptr, sizeof(int64_t) * (M->nrows + 1), kind));
  if (M->nnz > 0) {
    HIPX(hipMemcpy(H.col.data(), M->col, sizeof(int32_t) * M->nnz, kind));
    HIPX(hipMemcpy(H.val.data(), M->val, sizeof(double) * M->nnz, kind));
  }
  return check_structure(H.rowptr.data(), H.col.data(), H.nrows, H.ncols, M->nnz, name);
}

// transpose by counting sort on the column index (rows of the result keep
// increasing column order because the source rows are scanned in order)
HostCsr transpose(const HostCsr& M) {
  HostCsr T;
  T.nrows = M.ncols;
  T.ncols = M.nrows;
  T.rowptr.assign(T.nrows + 1, 0);
  const int64_t nnz = M.rowptr[M.nrows];
  T.col.resize(nnz);
  T.val.resize(nnz);
  for (int64_t k = 0; k < nnz; ++k) T.rowptr[M.col[k] + 1]++;
  for (int64_t j = 0; j < T.nrows; ++j) T.rowptr[j + 1] += T.rowptr[j];
  std::vector<int64_t> next(T.rowptr.begin(), T.rowptr.end() - 1);
  for (int64_t i = 0; i < M.nrows; ++i)
    for (int64_t k = M.rowptr[i]; k < M.rowptr[i + 1]; ++k) {
      const int64_t d = next[M.col[k]]++;
      T.col[d] = (int32_t)i;
      T.val[d] = M.val[k];
    }
  return T;
}

bool exactly_symmetric(const HostCsr& Q) {
  HostCsr T = transpose(Q);
  return T.rowptr == Q.rowptr && T.col == Q.col &&
         memcmp(T.val.data(), Q.val.data(), sizeof(double) * Q.val.size()) == 0;
}

struct HostPart {
  std::vector<int32_t> bounds, long_ptr, long_rows, tile_ptr, tiles;
  int32_t group = 1;
};

int pow2_ceil(double v) {
  int g = 1;
  while (g < v && g < 64) g <<= 1;
  return g;
}

// Row partition for nb workgroups over the rows of one or two matrices with
// the same rows (rp1, rp2: host row pointers, either may be null): contiguous
// ranges of near-equal work (entries + 2 per row); rows with more than
// kLongRow entries listed per workgroup; the other rows cut into tiles of at
// most tile_nnz_for(block) entries and tile_rows_for(block) rows, block being
// the workgroup size of the kernel that runs the partition (the LDS tile of
// its translation unit).  The lane group is the power of two at or above the
// mean length of the short rows.
// Tiles of the standalone product: runs of whole rows with at most
// spmv_stream_tile_nnz() entries and spmv_stream_tile_rows() rows; a row
// longer than that forms a tile of its own.  4 ints per tile: first row, end
// row, first entry, end entry.
std::vector<int32_t> stream_tiles(int64_t nrows, const int64_t* rp) {
  const int64_t cap = spmv_stream_tile_nnz(), rcap = spmv_stream_tile_rows();
  std::vector<int32_t> t;
  int64_t i = 0;
  while (i < nrows) {
    const int64_t start = i;
    if (rp[i + 1] - rp[i] > cap) {
      ++i;
    } else {
      while (i < nrows && i - start < rcap && rp[i + 1] - rp[start] <= cap) ++i;
    }
    const int32_t q[4] = {(int32_t)start, (int32_t)i, (int32_t)rp[start], (int32_t)rp[i]};
    t.insert(t.end(), q, q + 4);
  }
  return t;
}

HostPart build_part(int64_t nrows, int nb, const int64_t* rp1, const int64_t* rp2, int gscale = 0,
                    int block = kSolveBlock) {
  const int64_t tile_nnz = tile_nnz_for(block), tile_rows = tile_rows_for(block);
  HostPart P;
  auto len = [&](int64_t i) -> int64_t {
    return (rp1 ? rp1[i + 1] - rp1[i] : 0) + (rp2 ? rp2[i + 1] - rp2[i] : 0);
  };
  std::vector<int64_t> pref(nrows + 1, 0);
  int64_t short_nnz = 0, short_rows = 0;
  for (int64_t i = 0; i < nrows; ++i) {
    const int64_t l = len(i);
    pref[i + 1] = pref[i] + l + 2;
    if (l <= kLongRow) {
      short_nnz += l;
      short_rows++;
    }
  }
  P.bounds.resize(nb + 1);
  for (int b = 0; b <= nb; ++b) {
    const int64_t target = (int64_t)((double)pref[nrows] * b / nb);
    P.bounds[b] = (int32_t)(std::lower_bound(pref.begin(), pref.end(), target) - pref.begin());
    if (P.bounds[b] > nrows) P.bounds[b] = (int32_t)nrows;
  }
  P.bounds[0] = 0;
  P.bounds[nb] = (int32_t)nrows;
  for (int b = 1; b <= nb; ++b) P.bounds[b] = std::max(P.bounds[b], P.bounds[b - 1]);
  P.long_ptr.assign(nb + 1, 0);
  P.tile_ptr.assign(nb + 1, 0);
  int32_t ntiles = 0;
  for (int b = 0; b < nb; ++b) {
    int64_t i = P.bounds[b];
    const int64_t end = P.bounds[b + 1];
    while (i < end) {
      if (len(i) > kLongRow) {
        P.long_rows.push_back((int32_t)i);
        ++i;
        continue;
      }
      const int64_t start = i;
      int64_t acc = 0;
      while (i < end && len(i) <= kLongRow && acc + len(i) <= tile_nnz && i - start < tile_rows) {
        acc += len(i);
        ++i;
      }
      const int32_t t[6] = {(int32_t)start, (int32_t)i, (int32_t)(rp1 ? rp1[start] : 0), (int32_t)(rp1 ? rp1[i] : 0),
                            (int32_t)(rp2 ? rp2[start] : 0), (int32_t)(rp2 ? rp2[i] : 0)};
      P.tiles.insert(P.tiles.end(), t, t + 6);
      ++ntiles;
    }
    P.long_ptr[b + 1] = (int32_t)P.long_rows.size();
    P.tile_ptr[b + 1] = ntiles;
  }
  const double mean = short_rows ? (double)short_nnz / (double)short_rows : 1.0;
  P.group = pow2_ceil(mean);
  for (int k = 0; k < gscale && P.group < 64; ++k) P.group <<= 1;
  for (int k = 0; k > gscale && P.group > 1; --k) P.group >>= 1;
  return P;
}

}  // namespace

struct DevPart {
  int32_t* bounds = nullptr;
  int32_t* long_ptr = nullptr;
  int32_t* long_rows = nullptr;
  int32_t* tile_ptr = nullptr;
  int32_t* tiles = nullptr;
  int32_t group = 1;
  int64_t nlong = 0;
  Part view() const { return Part{bounds, long_ptr, long_rows, tile_ptr, tiles, group}; }
};

struct pdhcg_handle {
  int64_t n = 0, m = 0;
  int64_t nnzQ = 0, nnzA = 0;
  hipStream_t stream = nullptr;
  pdhcg_settings s{};
  int nb = 0;                 // workgroups of the persistent kernels
  double norm_A = 0.0, nb_inf = 0.0, nc_inf = 0.0, setup_s = 0.0, kkt_zero = 0.0;
  // device data
  int32_t *q_rowptr = nullptr, *q_col = nullptr, *a_rowptr = nullptr, *a_col = nullptr, *t_rowptr = nullptr,
          *t_col = nullptr;
  double *q_val = nullptr, *a_val = nullptr, *t_val = nullptr;
  float *q_val32 = nullptr, *a_val32 = nullptr, *t_val32 = nullptr;
  double *b = nullptr, *c = nullptr;
  double *x = nullptr, *y = nullptr, *xa = nullptr, *ya = nullptr, *ax = nullptr, *ax_avg = nullptr,
         *x_anc = nullptr, *y_anc = nullptr, *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
  float *x32 = nullptr, *xs32 = nullptr;
  float2* rp32 = nullptr;  // FP32 (r, p) records of the textbook CG
  double *r_alt = nullptr, *u0 = nullptr, *u1 = nullptr, *s0 = nullptr, *s1 = nullptr;
  double *x_prev = nullptr, *y_trial = nullptr, *ax_trial = nullptr;  // adaptive step size
  float4 *v32_0 = nullptr, *v32_1 = nullptr;   // interleaved FP32 (r, u, s) of the one-reduction CG
  double *part = nullptr, *tmp_x0 = nullptr, *tmp_y0 = nullptr, *scratch = nullptr;
  double* dscale = nullptr;  // D2 (n) then D1 (m) of the preconditioning; ones when off
  // Q = P P' + diag(d) given by a sparse P (pdhcg_create_lowrank): the Q
  // arrays then hold P (n x k), and P' (k x n) is stored beside it with a row
  // partition of its own
  int lowrank = 0;
  int64_t k = 0;
  int32_t *lt_rowptr = nullptr, *lt_col = nullptr;
  double *lt_val = nullptr, *lr_d = nullptr, *lr_pt = nullptr;
  float *lt_val32 = nullptr, *lr_pt32 = nullptr;
  DevPart plr;
  std::vector<int64_t> lrp_h;
  bool scaled = false;       // the device data are the preconditioned problem
  uint64_t* bar = nullptr;
  SolverState* st = nullptr;
  SolveParams* d_params = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  DevPart pn1, pcg, pm, pt;                // parts for the persistent kernels
  std::vector<int32_t> cg_bounds, m_bounds;          // host copies of the pcg / pm row ranges
  int cg_one_tile = 0;  // every workgroup's CG rows form one tile with no long row
  int64_t l2_bytes = 4 << 20;  // L2 of one XCD (device attribute at create)
  int res_bytes = 0;                                 // dynamic LDS of the last solve launch
  int32_t* stiles[3] = {nullptr, nullptr, nullptr};  // tiles of the standalone products (Q, A, A')
  int32_t nstiles[3] = {0, 0, 0};
  std::vector<void*> allocs;
  std::vector<double> c_host;  // c, for relKKT(0, 0) when b changes
  std::vector<int64_t> qrp_h, arp_h, trp_h;  // host row pointers, for re-planning
  int gscale = 0;              // lane-group scaling (log2) chosen by the autotuner
  int max_nb = 1;              // co-resident workgroups of the cooperative kernels at `threads`
  int threads = kSolveBlock;   // threads per workgroup of the cooperative kernels

  ~pdhcg_handle() {
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    for (void* p : allocs) (void)hipFree(p);
  }

  template <typename T>
  int alloc(T** p, int64_t count) {
    *p = nullptr;
    const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(PDHCG_ERR_OUT_OF_MEMORY,
                  "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    allocs.push_back(*p);
    return 0;
  }

  DevMat mat(int which) const {
    if (which == 0) return DevMat{(int32_t)n, (int32_t)(lowrank ? k : n), q_rowptr, q_col, q_val, q_val32};
    if (which == 1) return DevMat{(int32_t)m, (int32_t)n, a_rowptr, a_col, a_val, a_val32};
    return DevMat{(int32_t)n, (int32_t)m, t_rowptr, t_col, t_val, t_val32};
  }
};

namespace {

int upload_part(pdhcg_handle* h, const HostPart& H, DevPart& D) {
  int rc;
  if ((rc = h->alloc(&D.bounds, (int64_t)H.bounds.size()))) return rc;
  if ((rc = h->alloc(&D.long_ptr, (int64_t)H.long_ptr.size()))) return rc;
  if ((rc = h->alloc(&D.long_rows, (int64_t)H.long_rows.size()))) return rc;
  if ((rc = h->alloc(&D.tile_ptr, (int64_t)H.tile_ptr.size()))) return rc;
  if ((rc = h->alloc(&D.tiles, (int64_t)H.tiles.size()))) return rc;
  HIPX(hipMemcpyAsync(D.tile_ptr, H.tile_ptr.data(), sizeof(int32_t) * H.tile_ptr.size(), hipMemcpyHostToDevice,
                      h->stream));
  if (!H.tiles.empty())
    HIPX(hipMemcpyAsync(D.tiles, H.tiles.data(), sizeof(int32_t) * H.tiles.size(), hipMemcpyHostToDevice,
                        h->stream));
  HIPX(hipMemcpyAsync(D.bounds, H.bounds.data(), sizeof(int32_t) * H.bounds.size(), hipMemcpyHostToDevice, h->stream));
  HIPX(hipMemcpyAsync(D.long_ptr, H.long_ptr.data(), sizeof(int32_t) * H.long_ptr.size(), hipMemcpyHostToDevice,
                      h->stream));
  if (!H.long_rows.empty())
    HIPX(hipMemcpyAsync(D.long_rows, H.long_rows.data(), sizeof(int32_t) * H.long_rows.size(),
                        hipMemcpyHostToDevice, h->stream));
  D.group = H.group;
  D.nlong = (int64_t)H.long_rows.size();
  HIPX(hipStreamSynchronize(h->stream));
  return 0;
}

template <typename T>
int upload(pdhcg_handle* h, T* dst, const T* src, int64_t count) {
  if (count > 0) HIPX(hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyHostToDevice, h->stream));
  return 0;
}

int upload_csr(pdhcg_handle* h, const HostCsr& M, int32_t** rp, int32_t** col, double** val) {
  int rc;
  std::vector<int32_t> rp32(M.rowptr.begin(), M.rowptr.end());
  if ((rc = h->alloc(rp, M.nrows + 1))) return rc;
  if ((rc = h->alloc(col, (int64_t)M.col.size()))) return rc;
  if ((rc = h->alloc(val, (int64_t)M.val.size()))) return rc;
  if ((rc = upload(h, *rp, rp32.data(), M.nrows + 1))) return rc;
  if ((rc = upload(h, *col, M.col.data(), (int64_t)M.col.size()))) return rc;
  if ((rc = upload(h, *val, M.val.data(), (int64_t)M.val.size()))) return rc;
  HIPX(hipStreamSynchronize(h->stream));  // host vectors die at return
  return 0;
}

int ensure_mixed(pdhcg_handle* h) {
  int rc;
  if (h->q_val32) return 0;
  if ((rc = h->alloc(&h->q_val32, h->nnzQ))) return rc;
  if ((rc = h->alloc(&h->a_val32, h->nnzA))) return rc;
  if ((rc = h->alloc(&h->t_val32, h->nnzA))) return rc;
  if ((rc = h->alloc(&h->x32, h->n))) return rc;
  if ((rc = h->alloc(&h->rp32, h->n))) return rc;
  if ((rc = h->alloc(&h->xs32, std::max(h->n, h->m)))) return rc;
  if ((rc = h->alloc(&h->v32_0, h->n))) return rc;
  if ((rc = h->alloc(&h->v32_1, h->n))) return rc;
  HIPX(launch_to_f32(h->q_val, h->q_val32, h->nnzQ, h->stream));
  if (h->lowrank) {  // P' in FP32 for the products of the CG steps
    if ((rc = h->alloc(&h->lt_val32, h->nnzQ))) return rc;
    HIPX(launch_to_f32(h->lt_val, h->lt_val32, h->nnzQ, h->stream));
  }
  if (h->nnzA > 0) {
    HIPX(launch_to_f32(h->a_val, h->a_val32, h->nnzA, h->stream));
    HIPX(launch_to_f32(h->t_val, h->t_val32, h->nnzA, h->stream));
  }
  HIPX(hipStreamSynchronize(h->stream));
  return 0;
}

int check_settings(const pdhcg_settings* s) {
  if (!s) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null settings");
  if (!(s->tol_rel_kkt >= 0.0)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "tol_rel_kkt must be >= 0");
  if (s->max_iters < 0) return fail(PDHCG_ERR_INVALID_ARGUMENT, "max_iters must be >= 0");
  if (s->max_cg_iters < 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "max_cg_iters must be >= 1");
  if (s->cg_rule != 0 && s->cg_rule != 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "cg_rule must be 0 or 1");
  if (s->eval_period < 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "eval_period must be >= 1");
  if (!(s->primal_weight_init > 0.0)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "primal_weight_init must be > 0");
  if (!(s->step_eta_factor > 0.0)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "step_eta_factor must be > 0");
  if (s->power_iters < 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "power_iters must be >= 1");
  if (s->precision != 0 && s->precision != 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "precision must be 0 or 1");
  if (s->num_blocks < 0 || s->num_blocks > 4096) return fail(PDHCG_ERR_INVALID_ARGUMENT, "num_blocks out of range");
  if (s->cg_form < 0 || s->cg_form > 2) return fail(PDHCG_ERR_INVALID_ARGUMENT, "cg_form must be 0, 1 or 2");
  if (s->ruiz_iters < 0 || s->ruiz_iters > 100) return fail(PDHCG_ERR_INVALID_ARGUMENT, "ruiz_iters must be in [0, 100]");
  if (s->pock_chambolle != 0 && s->pock_chambolle != 1)
    return fail(PDHCG_ERR_INVALID_ARGUMENT, "pock_chambolle must be 0 or 1");
  if (s->step_rule != 0 && s->step_rule != 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "step_rule must be 0 or 1");
  if (s->threads != 0 && s->threads != 256 && s->threads != kSolveBlock)
    return fail(PDHCG_ERR_INVALID_ARGUMENT, "threads must be 0, 256 or 512");
  return 0;
}

void free_part(pdhcg_handle* h, DevPart& D) {
  for (int32_t** p : {&D.bounds, &D.long_ptr, &D.long_rows, &D.tile_ptr, &D.tiles}) {
    if (*p) {
      (void)hipFree(*p);
      h->allocs.erase(std::remove(h->allocs.begin(), h->allocs.end(), (void*)*p), h->allocs.end());
      *p = nullptr;
    }
  }
}

// (Re)build the partitions of the persistent kernels for nb workgroups and
// lane groups scaled by 2^gscale.
int plan_grid(pdhcg_handle* h, int nb, int gscale) {
  int rc;
  nb = std::max(1, std::min(nb, h->max_nb));
  h->nb = nb;
  h->gscale = gscale;
  const int64_t* qrp = h->qrp_h.data();
  const int64_t* arp = h->m ? h->arp_h.data() : nullptr;
  const int64_t* trp = h->m ? h->trp_h.data() : nullptr;
  for (DevPart* d : {&h->pn1, &h->pcg, &h->pm, &h->pt, &h->plr}) free_part(h, *d);
  if ((rc = upload_part(h, build_part(h->n, nb, qrp, trp, gscale, h->threads), h->pn1))) return rc;
  const HostPart pcg = build_part(h->n, nb, qrp, nullptr, gscale, h->threads);
  const HostPart pm = build_part(h->m, nb, arp, nullptr, gscale, h->threads);
  h->cg_bounds = pcg.bounds;
  h->m_bounds = pm.bounds;
  h->cg_one_tile = 1;
  for (int b = 0; b < nb; ++b)
    if (pcg.tile_ptr[b + 1] - pcg.tile_ptr[b] != 1 || pcg.long_ptr[b + 1] != pcg.long_ptr[b]) h->cg_one_tile = 0;
  if ((rc = upload_part(h, pcg, h->pcg))) return rc;
  if ((rc = upload_part(h, pm, h->pm))) return rc;
  if ((rc = upload_part(h, build_part(h->n, nb, trp, nullptr, gscale, h->threads), h->pt))) return rc;
  if (h->lowrank && (rc = upload_part(h, build_part(h->k, nb, h->lrp_h.data(), nullptr, gscale, h->threads), h->plr)))
    return rc;
  return 0;
}

// Threads per workgroup of the cooperative kernels: the setting, else 256
// (two workgroups per CU that wait apart, at twice the arrivals per grid
// barrier) once the gathered vectors stream from the last-level cache (the
// textbook CG's FP32 (r, p) records and the FP32 x, 12 n bytes, beyond the
// L2 of one XCD), and 512 below that size or for a low-rank Q.  Random QPs
// to 1e-4, 512 against 256 threads: n = 3e5 160 ms / 167 ms, n = 6e5
// 324 / 310 ms, n = 1e6 1 717 / 1 622 ms; power-law QP n = 2e6: 654 / 606 ms.
int solve_threads(const pdhcg_handle* h, const pdhcg_settings& s) {
  if (s.threads) return s.threads;
  return (!h->lowrank && 12 * h->n > h->l2_bytes) ? 256 : kSolveBlock;
}

// the co-resident workgroups of the cooperative kernels at h->threads
int set_max_nb(pdhcg_handle* h) {
  int dev = 0, cus = 0, per_cu = 0;
  HIPX(hipGetDevice(&dev));
  HIPX(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIPX(solve_occupancy(h->threads, &per_cu));
  h->max_nb = std::max(1, std::min(cus * std::max(per_cu, 1), 1024));
  return 0;
}

// The planner's grid: about a thousand work units per workgroup, below which
// the grid barrier outweighs the work it spreads (n = 1000 random QP: 64
// workgroups 65 ms, 16 70 ms, 128 69 ms per solve), up to one 512-thread or
// two 256-thread workgroups per CU of 256.
int default_nb(const pdhcg_handle* h) {
  const double work = (double)h->nnzQ + 0.25 * (double)h->nnzA + (double)(h->n + h->m);
  const int cap = 256 * (kSolveBlock / h->threads);
  int nb = 8;
  while (nb < cap && work / nb > 1024.0) nb <<= 1;
  return nb;
}

int plan(pdhcg_handle* h, const HostCsr& Q, const HostCsr& A, const HostCsr& T) {
  int rc;
  int dev = 0, l2 = 0;
  HIPX(hipGetDevice(&dev));
  HIPX(hipDeviceGetAttribute(&l2, hipDeviceAttributeL2CacheSize, dev));
  if (l2 > 0) h->l2_bytes = l2;
  h->threads = solve_threads(h, h->s);
  if ((rc = set_max_nb(h))) return rc;
  const int nb = h->s.num_blocks ? h->s.num_blocks : default_nb(h);
  h->qrp_h = Q.rowptr;
  if (A.nrows) {
    h->arp_h = A.rowptr;
    h->trp_h = T.rowptr;
  }
  const int64_t* qrp = Q.rowptr.data();
  const int64_t* arp = A.nrows ? A.rowptr.data() : nullptr;
  const int64_t* trp = A.nrows ? T.rowptr.data() : nullptr;
  if ((rc = plan_grid(h, nb, 0))) return rc;
  // standalone products: one short tile per workgroup
  const int64_t* rps[3] = {qrp, arp, trp};
  const int64_t nrs[3] = {h->n, h->m, h->n};
  for (int k = 0; k < 3; ++k) {
    if (!rps[k] || nrs[k] == 0) continue;
    const std::vector<int32_t> t = stream_tiles(nrs[k], rps[k]);
    h->nstiles[k] = (int32_t)(t.size() / 4);
    if ((rc = h->alloc(&h->stiles[k], (int64_t)t.size()))) return rc;
    HIPX(hipMemcpyAsync(h->stiles[k], t.data(), sizeof(int32_t) * t.size(), hipMemcpyHostToDevice, h->stream));
  }
  HIPX(hipStreamSynchronize(h->stream));
  return 0;
}

// LDS use of the solve kernel for this launch, in this order while it fits
// the LDS a workgroup can have beside the kernel's static LDS with nb
// workgroups co-resident: the CG state of the workgroup's CG rows (five FP64
// values per row), the CG rows of Q, the dual rows of A (each sized by the
// largest workgroup block).
int plan_residency(pdhcg_handle* h, SolveParams& p) {
  p.res_cg = p.res_m = 0;
  p.res_vbytes = h->s.precision == 1 ? 4 : 8;
  p.res_m_off = 0;
  p.own_cg = p.own_off = p.cg_chain = 0;
  p.cg_own = nullptr;
  h->res_bytes = 0;
  int dev = 0, cus = 0, lds_cu = 0, stat = 0;
  HIPX(hipGetDevice(&dev));
  HIPX(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIPX(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
  HIPX(solve_kernel_lds(h->threads, &stat));
  const int per_cu = (h->nb + cus - 1) / std::max(cus, 1);
  const int64_t budget = (int64_t)lds_cu / std::max(per_cu, 1) - stat - 256;
  auto block = [&](const std::vector<int32_t>& bnd, const std::vector<int64_t>& rp) {
    int64_t best = 0;
    for (size_t b = 0; b + 1 < bnd.size(); ++b)
      best = std::max(best, res_block_bytes(bnd[b + 1] - bnd[b], rp[bnd[b + 1]] - rp[bnd[b]], p.res_vbytes));
    return best;
  };
  int64_t bo = 0;
  for (size_t b = 0; b + 1 < h->cg_bounds.size(); ++b)
    bo = std::max(bo, align16(5 * 8 * (int64_t)(h->cg_bounds[b + 1] - h->cg_bounds[b])));
  const int64_t bq = block(h->cg_bounds, h->qrp_h);
  const int64_t ba = h->m ? block(h->m_bounds, h->arp_h) : 0;
  int64_t total = 0;
  // (the adaptive step size gathers the FP64 x of every row after the primal
  // step, so the CG state then stays in device memory)
  if (p.u0 && bo > 0 && bo <= budget && !h->s.step_rule) {
    p.own_cg = 1;
    total = bo;
  }
  if (!h->lowrank && total + bq <= budget) {  // (a low-rank Q's products gather t, not p)
    p.res_cg = 1;
    total += bq;
  }
  if (h->m && total + ba <= budget) {
    p.res_m = 1;
    total += ba;
  }
  // layout: Q block at 0, then the A block, then the CG state
  const int64_t q_end = p.res_cg ? bq : 0;
  p.res_m_off = (int32_t)q_end;
  p.own_off = (int32_t)(q_end + (p.res_m ? ba : 0));
  if (total > 0) {
    int occ = 0;
    HIPX(solve_occupancy_dyn(h->threads, (int)total, &occ));
    if (occ * cus < h->nb) {  // would break co-residency: keep everything in device memory
      p.res_cg = p.res_m = p.own_cg = 0;
      total = 0;
    }
  }
  // the chained CG steps (every workgroup or none: they take the CG decisions
  // themselves, so all must run the same code)
  p.cg_chain = p.own_cg && p.res_cg && p.res_vbytes == 4 && h->cg_one_tile;
  h->res_bytes = (int)total;
  return 0;
}

SolveParams make_params(pdhcg_handle* h) {
  SolveParams p{};
  p.Q = h->mat(0);
  p.A = h->mat(1);
  p.At = h->mat(2);
  p.b = h->b;
  p.c = h->c;
  p.n = (int32_t)h->n;
  p.m = (int32_t)h->m;
  p.x = h->x; p.y = h->y; p.xa = h->xa; p.ya = h->ya; p.ax = h->ax; p.ax_avg = h->ax_avg;
  p.x_anc = h->x_anc; p.y_anc = h->y_anc; p.r = h->r; p.p0 = h->p0; p.p1 = h->p1; p.q = h->q;
  p.x32 = h->x32; p.rp32 = h->rp32;
  p.r_alt = h->r_alt; p.u0 = h->u0; p.u1 = h->u1; p.s0 = h->s0; p.s1 = h->s1;
  p.v32_0 = h->v32_0; p.v32_1 = h->v32_1;
  // CG form: the single-reduction steps gather 16 bytes per column (FP32 r, u,
  // s), the textbook steps 8 (the FP32 (r, p) record) at one more grid barrier per step;
  // the first wins while the gathered vector stays in an XCD's L2, the second
  // once the gathers stream from the last-level cache
  // (a low-rank Q takes the textbook form: its products need t = P' p first)
  const bool single = !h->lowrank && (h->s.cg_form == 1 || (h->s.cg_form == 0 && 16 * h->n <= h->l2_bytes));
  if (!single) {
    p.u0 = nullptr;
    p.v32_0 = p.v32_1 = nullptr;
  }
  p.part = h->part;
  p.bar = h->bar;
  p.st = h->st;
  p.pn1 = h->pn1.view();
  p.pcg = h->pcg.view();
  p.pm = h->pm.view();
  p.pt = h->pt.view();
  if (h->lowrank) {
    p.Lt = DevMat{(int32_t)h->k, (int32_t)h->n, h->lt_rowptr, h->lt_col, h->lt_val, h->lt_val32, 0, 0};
    p.plr = h->plr.view();
    p.lr_d = h->lr_d;
    p.lr_pt = h->lr_pt;
    p.lr_pt32 = h->lr_pt32;
  }
  p.nb_inf = h->nb_inf;
  p.nc_inf = h->nc_inf;
  p.dn = h->scaled ? h->dscale : nullptr;
  p.dm = h->scaled && h->m > 0 ? h->dscale + h->n : nullptr;
  const pdhcg_settings& s = h->s;
  p.tol = s.tol_rel_kkt;
  p.eps_factor = s.cg_eps_factor;
  p.beta_suf = s.beta_sufficient;
  p.beta_nec = s.beta_necessary;
  p.beta_art = s.beta_artificial;
  p.theta = s.primal_weight_theta;
  p.max_iters = s.max_iters;
  p.iters_this_launch = 5000;
  p.time_limit_ticks = s.time_limit_s > 0.0 ? (uint64_t)(s.time_limit_s * 1e8) : 0;  // 100 MHz clock
  p.max_cg = s.max_cg_iters;
  p.cg_rule = s.cg_rule;
  p.restart_to = s.restart_to;
  p.eval_period = s.eval_period;
  p.mixed_allowed = s.precision == 1;
  p.step_rule = s.step_rule;
  if (s.step_rule) {
    p.x_prev = h->x_prev;
    p.y_trial = h->y_trial;
    p.ax_trial = h->ax_trial;
  }
  return p;
}

int estimate_norm(pdhcg_handle* h) {
  if (h->m == 0 || h->nnzA == 0) {
    h->norm_A = 0.0;
    return 0;
  }
  PowerParams pp{};
  pp.A = h->mat(1);
  pp.At = h->mat(2);
  pp.v = h->p0;
  pp.w = h->p1;
  pp.u = h->ax_avg;
  pp.part = h->part;
  pp.bar = h->bar;
  pp.out = h->scratch;
  pp.pn = h->pt.view();
  pp.pm = h->pm.view();
  pp.iters = h->s.power_iters;
  HIPX(hipMemsetAsync(h->bar, 0, sizeof(uint64_t) * kBarWords, h->stream));
  HIPX(launch_power(h->threads, pp, h->nb, h->stream));
  double v = 0.0;
  uint64_t abort_word = 0;
  HIPX(hipMemcpyAsync(&v, h->scratch, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipMemcpyAsync(&abort_word, h->bar + kBarAbortWord, sizeof(uint64_t), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  if (abort_word != 0) return fail(PDHCG_ERR_HIP, "grid barrier of the power iteration timed out");
  h->norm_A = v;
  return 0;
}

}  // namespace

extern "C" {

void pdhcg_default_settings(pdhcg_settings* s) {
  if (!s) return;
  memset(s, 0, sizeof(*s));
  s->tol_rel_kkt = 1e-4;
  s->max_iters = 100000;
  s->max_cg_iters = 100;
  s->cg_rule = 0;
  s->cg_eps_factor = 0.05;
  s->beta_sufficient = 0.2;
  s->beta_necessary = 0.8;
  s->beta_artificial = 0.2;
  s->restart_to = 0;
  s->eval_period = 64;
  s->primal_weight_theta = 0.2;
  s->primal_weight_init = 1.0;
  s->step_eta_factor = 0.5;
  s->power_iters = 100;
  s->precision = 0;
  s->time_limit_s = 0.0;
  s->num_blocks = 0;
  s->warm_fallback = 1;
  s->verbose = 0;
  s->cg_form = 0;
  s->ruiz_iters = 0;
  s->pock_chambolle = 0;
  s->step_rule = 0;
  s->threads = 0;
}

}  // extern "C"

namespace {

// pdhcg_create, and pdhcg_create_lowrank when lowrank is set (Qc is then P,
// n x k, and d the diagonal, NULL for zero)
int create_impl(pdhcg_handle** out, const pdhcg_csr* Qc, const pdhcg_csr* Ac, const double* b, const double* c,
                int32_t vec_on_device, const pdhcg_settings* s, void* hip_stream, bool lowrank, const double* d) {
  const double t0 = now_s();
  if (!out) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle pointer");
  *out = nullptr;
  int rc;
  if ((rc = check_settings(s))) return rc;
  HostCsr Q, A;
  if ((rc = fetch_csr(Qc, Q, lowrank ? "P" : "Q"))) return rc;
  if ((rc = fetch_csr(Ac, A, "A"))) return rc;
  if (A.ncols != Q.nrows) return fail(PDHCG_ERR_INVALID_ARGUMENT, "A must have as many columns as Q");
  if (Q.nrows == 0) return fail(PDHCG_ERR_INVALID_ARGUMENT, "n must be >= 1");
  if (!lowrank) {
    if (Q.nrows != Q.ncols) return fail(PDHCG_ERR_INVALID_ARGUMENT, "Q must be square");
    if (!exactly_symmetric(Q)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "Q is not exactly symmetric");
  } else {
    if (Q.ncols < 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "P must have k >= 1 columns");
    if (s->ruiz_iters != 0 || s->pock_chambolle != 0)
      return fail(PDHCG_ERR_INVALID_ARGUMENT, "a low-rank Q takes no diagonal preconditioning");
    if (s->step_rule != 0)
      return fail(PDHCG_ERR_INVALID_ARGUMENT, "a low-rank Q takes the constant step rule (step_rule = 0)");
  }
  if (!c || (A.nrows > 0 && !b)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null b or c");
  std::vector<double> hd;
  if (lowrank) {
    hd.assign(Q.nrows, 0.0);
    if (d && hipMemcpy(hd.data(), d, sizeof(double) * Q.nrows,
                       vec_on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost) != hipSuccess)
      return fail(PDHCG_ERR_HIP, "copy of d failed");
    for (double v : hd)
      if (!(v >= 0.0) || std::isinf(v)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "d must be finite and >= 0");
  }
  HostCsr T = transpose(A);

  pdhcg_handle* h = new pdhcg_handle();
  h->lowrank = lowrank ? 1 : 0;
  h->n = Q.nrows;
  h->m = A.nrows;
  h->nnzQ = (int64_t)Q.col.size();
  h->nnzA = (int64_t)A.col.size();
  h->stream = (hipStream_t)hip_stream;
  h->s = *s;
  auto bail = [&](int code) {
    delete h;
    return code;
  };
  std::vector<double> hb(h->m), hc(h->n);
  hipMemcpyKind kind = vec_on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost;
  if (h->m > 0 && hipMemcpy(hb.data(), b, sizeof(double) * h->m, kind) != hipSuccess)
    return bail(fail(PDHCG_ERR_HIP, "copy of b failed"));
  if (hipMemcpy(hc.data(), c, sizeof(double) * h->n, kind) != hipSuccess)
    return bail(fail(PDHCG_ERR_HIP, "copy of c failed"));
  h->nb_inf = max_abs_nan(hb.data(), h->m);
  h->nc_inf = max_abs_nan(hc.data(), h->n);
  h->kkt_zero = kkt_at_zero(hb.data(), h->m, hc.data(), h->n);
  h->c_host = hc;

  if ((rc = upload_csr(h, Q, &h->q_rowptr, &h->q_col, &h->q_val))) return bail(rc);
  if ((rc = upload_csr(h, A, &h->a_rowptr, &h->a_col, &h->a_val))) return bail(rc);
  if ((rc = upload_csr(h, T, &h->t_rowptr, &h->t_col, &h->t_val))) return bail(rc);
  if (lowrank) {  // P' beside P, d, and t = P' v (FP64 and an FP32 copy)
    const HostCsr Lt = transpose(Q);
    h->k = Q.ncols;
    h->lrp_h = Lt.rowptr;
    if ((rc = upload_csr(h, Lt, &h->lt_rowptr, &h->lt_col, &h->lt_val))) return bail(rc);
    if ((rc = h->alloc(&h->lr_d, h->n))) return bail(rc);
    if ((rc = h->alloc(&h->lr_pt, h->k))) return bail(rc);
    if ((rc = h->alloc(&h->lr_pt32, h->k))) return bail(rc);
    if ((rc = upload(h, h->lr_d, hd.data(), h->n))) return bail(rc);
  }
  const int64_t n = h->n, m = h->m;
  double** nvecs[] = {&h->c, &h->x, &h->xa, &h->x_anc, &h->r, &h->p0, &h->p1, &h->q, &h->tmp_x0,
                      &h->r_alt, &h->u0, &h->u1, &h->s0, &h->s1, &h->x_prev};
  for (double** v : nvecs)
    if ((rc = h->alloc(v, n))) return bail(rc);
  double** mvecs[] = {&h->b, &h->y, &h->ya, &h->ax, &h->ax_avg, &h->y_anc, &h->tmp_y0, &h->y_trial, &h->ax_trial};
  for (double** v : mvecs)
    if ((rc = h->alloc(v, m))) return bail(rc);
  if ((rc = h->alloc(&h->scratch, 16))) return bail(rc);
  if ((rc = h->alloc(&h->part, (int64_t)NSLOT * 4096))) return bail(rc);
  if ((rc = h->alloc(&h->bar, kBarWords))) return bail(rc);
  if ((rc = h->alloc(&h->st, 1))) return bail(rc);
  if ((rc = h->alloc(&h->d_params, 1))) return bail(rc);
  if ((rc = upload(h, h->b, hb.data(), m))) return bail(rc);
  if ((rc = upload(h, h->c, hc.data(), n))) return bail(rc);
  if ((rc = h->alloc(&h->dscale, n + m))) return bail(rc);
  {
    const std::vector<double> ones(n + m, 1.0);
    if ((rc = upload(h, h->dscale, ones.data(), n + m))) return bail(rc);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(PDHCG_ERR_HIP, "stream sync failed"));
  }
  if (s->ruiz_iters > 0 || s->pock_chambolle) {
    // preconditioning (Sec. 4, preprocessing): scale Q, A, A', b, c on the
    // device; relKKT stays that of the caller's problem, so the norms of b and
    // c and relKKT(0, 0) keep the values taken above from the unscaled data
    double* f = nullptr;
    if ((rc = h->alloc(&f, n + m))) return bail(rc);
    if (launch_precondition(h->mat(0), h->mat(1), h->mat(2), h->nnzQ, h->nnzA, s->ruiz_iters, s->pock_chambolle, f,
                            h->dscale, h->dscale + n, h->stream) != hipSuccess ||
        launch_diag(h->b, h->dscale + n, m, 0, h->b, h->stream) != hipSuccess ||
        launch_diag(h->c, h->dscale, n, 0, h->c, h->stream) != hipSuccess)
      return bail(fail(PDHCG_ERR_HIP, "preconditioning kernels failed to launch"));
    if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(PDHCG_ERR_HIP, "preconditioning failed"));
    h->scaled = true;
  }
  if ((rc = plan(h, Q, A, T))) return bail(rc);
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess)
    return bail(fail(PDHCG_ERR_HIP, "hipEventCreate failed"));
  if (s->precision == 1 && (rc = ensure_mixed(h))) return bail(rc);
  if ((rc = estimate_norm(h))) return bail(rc);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(PDHCG_ERR_HIP, "stream sync failed"));
  h->setup_s = now_s() - t0;
  if (s->verbose && lowrank) fprintf(stderr, "[pdhcg] low-rank Q = P P' + diag(d), k=%lld\n", (long long)h->k);
  if (s->verbose)
    fprintf(stderr,
            "[pdhcg] n=%lld m=%lld nnzQ=%lld nnzA=%lld nb=%d x %d threads groups n1=%d q=%d m=%d ||A||=%.6g "
            "setup=%.3fs\n",
            (long long)n, (long long)m, (long long)h->nnzQ, (long long)h->nnzA, h->nb, h->threads, h->pn1.group,
            h->pcg.group,
            h->pm.group, h->norm_A, h->setup_s);
  *out = h;
  return 0;
}

}  // namespace

extern "C" {

int pdhcg_create(pdhcg_handle** out, const pdhcg_csr* Qc, const pdhcg_csr* Ac, const double* b, const double* c,
                 int32_t vec_on_device, const pdhcg_settings* s, void* hip_stream) {
  return create_impl(out, Qc, Ac, b, c, vec_on_device, s, hip_stream, false, nullptr);
}

int pdhcg_create_lowrank(pdhcg_handle** out, const pdhcg_csr* P, const double* d, const pdhcg_csr* Ac,
                         const double* b, const double* c, int32_t vec_on_device, const pdhcg_settings* s,
                         void* hip_stream) {
  return create_impl(out, P, Ac, b, c, vec_on_device, s, hip_stream, true, d);
}

int pdhcg_set_settings(pdhcg_handle* h, const pdhcg_settings* s) {
  if (!h) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle");
  int rc;
  if ((rc = check_settings(s))) return rc;
  if (h->lowrank && s->step_rule != 0)
    return fail(PDHCG_ERR_INVALID_ARGUMENT, "a low-rank Q takes the constant step rule (step_rule = 0)");
  if (s->ruiz_iters != h->s.ruiz_iters || s->pock_chambolle != h->s.pock_chambolle)
    return fail(PDHCG_ERR_INVALID_ARGUMENT, "ruiz_iters and pock_chambolle are fixed at pdhcg_create");
  const int threads = solve_threads(h, *s);
  const bool replan = (s->num_blocks != 0 && s->num_blocks != h->nb) || threads != h->threads;
  const int32_t old_power = h->s.power_iters;
  h->s = *s;
  if (threads != h->threads) {  // other kernels: their co-residency and tile sizes
    h->threads = threads;
    if ((rc = set_max_nb(h))) return rc;
  }
  if (replan && (rc = plan_grid(h, s->num_blocks ? s->num_blocks : default_nb(h), h->gscale))) return rc;
  if (s->precision == 1 && (rc = ensure_mixed(h))) return rc;
  if (s->power_iters != old_power && (rc = estimate_norm(h))) return rc;
  return 0;
}

int pdhcg_set_b(pdhcg_handle* h, const double* b, int32_t vec_on_device) {
  if (!h || (h->m > 0 && !b)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle or b");
  std::vector<double> hb(h->m);
  if (h->m > 0) {
    HIPX(hipMemcpy(hb.data(), b, sizeof(double) * h->m, vec_on_device ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
    HIPX(hipMemcpyAsync(h->b, hb.data(), sizeof(double) * h->m, hipMemcpyHostToDevice, h->stream));
    if (h->scaled) HIPX(launch_diag(h->b, h->dscale + h->n, h->m, 0, h->b, h->stream));  // b~ = D1 b
    HIPX(hipStreamSynchronize(h->stream));
  }
  h->nb_inf = max_abs_nan(hb.data(), h->m);
  h->kkt_zero = kkt_at_zero(hb.data(), h->m, h->c_host.data(), h->n);
  return 0;
}

int pdhcg_solve(pdhcg_handle* h, const double* x0, const double* y0, double* x_out, double* y_out,
                int32_t vec_on_device, pdhcg_result* res) {
  if (!h) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle");
  if (!x_out || (h->m > 0 && !y_out)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null output");
  const double t0 = now_s();
  int rc;
  if (h->s.precision == 1 && (rc = ensure_mixed(h))) return rc;
  const double* dx0 = nullptr;
  const double* dy0 = nullptr;
  hipMemcpyKind in_kind = vec_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  if (x0) {
    HIPX(hipMemcpyAsync(h->tmp_x0, x0, sizeof(double) * h->n, in_kind, h->stream));
    if (h->scaled) HIPX(launch_diag(h->tmp_x0, h->dscale, h->n, 1, h->tmp_x0, h->stream));  // x~ = x / D2
    dx0 = h->tmp_x0;
  }
  if (y0 && h->m > 0) {
    HIPX(hipMemcpyAsync(h->tmp_y0, y0, sizeof(double) * h->m, in_kind, h->stream));
    if (h->scaled) HIPX(launch_diag(h->tmp_y0, h->dscale + h->n, h->m, 1, h->tmp_y0, h->stream));  // y~ = y / D1
    dy0 = h->tmp_y0;
  }
  SolveParams p = make_params(h);
  if ((rc = plan_residency(h, p))) return rc;
  p.x0 = dx0;
  p.y0 = dy0;
  p.kkt_zero = (h->s.warm_fallback && (dx0 || dy0)) ? h->kkt_zero : 0.0;
  SolverState st{};
  st.K_anchor = std::numeric_limits<double>::quiet_NaN();
  st.K_prev = std::numeric_limits<double>::infinity();
  st.omega = h->s.primal_weight_init;
  st.eta = h->s.step_eta_factor / (h->norm_A > 0.0 ? h->norm_A : 1.0);
  st.tau = st.eta / st.omega;
  st.sigma = st.eta * st.omega;
  st.norm_A = h->norm_A;
  st.mixed = h->s.precision == 1 ? 1 : 0;
  HIPX(hipMemcpyAsync(h->st, &st, sizeof(st), hipMemcpyHostToDevice, h->stream));
  HIPX(hipMemcpyAsync(h->d_params, &p, sizeof(p), hipMemcpyHostToDevice, h->stream));
  HIPX(launch_init_point(h->d_params, h->n, h->m, h->stream));
  double kernel_ms = 0.0;
  for (;;) {
    HIPX(hipMemsetAsync(h->bar, 0, sizeof(uint64_t) * kBarWords, h->stream));
    HIPX(hipEventRecord(h->ev0, h->stream));
    HIPX(launch_solve(h->threads, h->d_params, h->nb, h->res_bytes, h->stream));
    HIPX(hipEventRecord(h->ev1, h->stream));
    HIPX(hipMemcpyAsync(&st, h->st, sizeof(st), hipMemcpyDeviceToHost, h->stream));
    HIPX(hipStreamSynchronize(h->stream));
    float ms = 0.0f;
    HIPX(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    kernel_ms += ms;
    if (h->s.verbose)
      fprintf(stderr, "[pdhcg] iters=%lld cg=%lld restarts=%lld omega=%.4g done=%d\n", (long long)st.k_total,
              (long long)st.cg_total, (long long)st.restarts, st.omega, st.done);
    if (st.done != 0) break;
  }
  if (st.done < 0) return fail(PDHCG_ERR_HIP, "grid barrier timed out in the solve kernel");
  hipMemcpyKind out_kind = vec_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const double* xr = h->x;
  const double* yr = h->y;
  if (h->scaled) {  // x = D2 x~, y = D1 y~ (the start-point buffers are free again)
    HIPX(launch_diag(h->x, h->dscale, h->n, 0, h->tmp_x0, h->stream));
    HIPX(launch_diag(h->y, h->dscale + h->n, h->m, 0, h->tmp_y0, h->stream));
    xr = h->tmp_x0;
    yr = h->tmp_y0;
  }
  HIPX(hipMemcpyAsync(x_out, xr, sizeof(double) * h->n, out_kind, h->stream));
  if (h->m > 0) HIPX(hipMemcpyAsync(y_out, yr, sizeof(double) * h->m, out_kind, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  if (res) {
    res->status = st.status;
    res->returned_average = st.returned_average;
    res->rel_primal = st.r_p;
    res->rel_dual = st.r_d;
    res->rel_gap = st.r_g;
    res->rel_kkt = st.kkt;
    res->primal_obj = st.pobj;
    res->dual_obj = st.dobj;
    res->iters = st.k_total;
    res->cg_iters_total = st.cg_total;
    res->restarts = st.restarts;
    res->norm_A = h->norm_A;
    res->setup_s = h->setup_s;
    res->solve_s = now_s() - t0;
    res->kernel_s = kernel_ms * 1e-3;
    res->kkt_evals = st.evals;
    res->cold_fallback = st.cold_fallback;
    res->rejected_steps = st.rejections;
    res->qx_formed = st.qx_formed;
    res->step_eta = st.eta;
  }
  return 0;
}

int pdhcg_get_scaling(const pdhcg_handle* h, double* d1_out, double* d2_out, int32_t vec_on_device) {
  if (!h || !d2_out || (h->m > 0 && !d1_out)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle or output");
  const hipMemcpyKind kind = vec_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIPX(hipMemcpyAsync(d2_out, h->dscale, sizeof(double) * h->n, kind, h->stream));
  if (h->m > 0) HIPX(hipMemcpyAsync(d1_out, h->dscale + h->n, sizeof(double) * h->m, kind, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  return 0;
}

int pdhcg_spmv(pdhcg_handle* h, int32_t which, int32_t precision, const double* x, double* y, int32_t repeats) {
  if (!h || !x || !y) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null argument");
  if (which < 0 || which > 2) return fail(PDHCG_ERR_INVALID_ARGUMENT, "which must be 0 (Q), 1 (A) or 2 (A')");
  if (precision != 0 && precision != 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "precision must be 0 or 1");
  if (which == 0 && h->lowrank)
    return fail(PDHCG_ERR_INVALID_ARGUMENT, "a low-rank handle holds P, not Q: which must be 1 or 2");
  int rc;
  if (precision == 1 && (rc = ensure_mixed(h))) return rc;
  const DevMat M = h->mat(which);
  if (M.nrows == 0) return 0;
  float* x32 = nullptr;
  if (precision == 1) {
    x32 = h->xs32;  // scratch FP32 copy of x
    HIPX(launch_to_f32(x, x32, M.ncols, h->stream));
  }
  for (int r = 0; r < std::max(repeats, 1); ++r)
    HIPX(launch_spmv_stream(M.rowptr, M.col, M.val, M.val32, precision, x, x32, y, h->stiles[which],
                            h->nstiles[which], h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  return 0;
}

int pdhcg_autotune(pdhcg_handle* h, int32_t iters, int32_t* num_blocks, int32_t* group_scale) {
  if (!h) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle");
  if (iters < 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "iters must be >= 1");
  int rc;
  double* xs = nullptr;
  double* ys = nullptr;
  if ((rc = h->alloc(&xs, h->n))) return rc;
  if ((rc = h->alloc(&ys, std::max<int64_t>(h->m, 1)))) return rc;
  const pdhcg_settings saved = h->s;
  h->s.tol_rel_kkt = 0.0;
  h->s.max_iters = iters;
  h->s.time_limit_s = 0.0;
  h->s.verbose = 0;
  double best = 1e300;
  int best_nb = h->nb, best_g = h->gscale, best_t = h->threads;
  for (int t : {kSolveBlock, 256}) {
    h->threads = t;
    if ((rc = set_max_nb(h))) break;
    for (int nb : {64, 128, 256, 512}) {
      if (nb > h->max_nb) continue;
      for (int g : {-1, 0, 1}) {
        if ((rc = plan_grid(h, nb, g))) break;
        pdhcg_result r;
        if ((rc = pdhcg_solve(h, nullptr, nullptr, xs, ys, 1, &r))) break;
        const double per = r.kernel_s / (double)std::max<int64_t>(r.iters, 1);
        if (per < best) {
          best = per;
          best_nb = h->nb;
          best_g = g;
          best_t = t;
        }
      }
      if (rc) break;
    }
    if (rc) break;
  }
  h->s = saved;
  // the best plan found so far, also after a failed candidate
  h->threads = best_t;
  int rc_plan = set_max_nb(h);
  if (!rc_plan) rc_plan = plan_grid(h, best_nb, best_g);
  for (double* p : {xs, ys}) {
    (void)hipFree(p);
    h->allocs.erase(std::remove(h->allocs.begin(), h->allocs.end(), (void*)p), h->allocs.end());
  }
  if (rc) return rc;
  if (rc_plan) return rc_plan;
  h->s.num_blocks = best_nb;
  h->s.threads = best_t;
  if (num_blocks) *num_blocks = best_nb;
  if (group_scale) *group_scale = best_g;
  return 0;
}

int pdhcg_plan_info(const pdhcg_handle* h, int32_t* num_blocks, int32_t* group_n, int32_t* group_q, int32_t* group_m,
                    int64_t* long_rows, int32_t* threads) {
  if (!h) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle");
  if (num_blocks) *num_blocks = h->nb;
  if (group_n) *group_n = h->pn1.group;
  if (group_q) *group_q = h->pcg.group;
  if (group_m) *group_m = h->pm.group;
  if (long_rows) *long_rows = h->pn1.nlong + h->pcg.nlong + h->pm.nlong;
  if (threads) *threads = h->threads;
  return 0;
}

void pdhcg_destroy(pdhcg_handle* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

const char* pdhcg_error_string(int code) {
  switch (code) {
    case PDHCG_OK: return "ok";
    case PDHCG_ERR_INVALID_ARGUMENT: return "invalid argument";
    case PDHCG_ERR_OUT_OF_MEMORY: return "out of device memory";
    case PDHCG_ERR_HIP: return "HIP error";
    default: return "unknown error";
  }
}

const char* pdhcg_last_error(void) { return g_err.c_str(); }

}  // extern "C"


namespace {

// host-side bookkeeping of one QP of a batch: offsets into the packed arrays
struct BatchInst {
  int32_t n = 0, m = 0;
  int32_t dense = 0;
  int32_t q_rank = 0;  // k of a factored Q (dense = 2)
  // row partitions per workgroup size (index 0: 256 threads, 1: 512; the
  // second only for a handle the autotuner may switch): offset into the
  // packed lists, lane groups of the four partitions (n-side, CG, A, A')
  int32_t g[2][4] = {{1, 1, 1, 1}, {1, 1, 1, 1}};
  int32_t x0_given = 0, y0_given = 0;
  int64_t q_rp = 0, q_nz = 0, a_rp = 0, a_nz = 0, t_rp = 0, t_nz = 0;
  int64_t voff_n = 0, voff_m = 0;
  int64_t part_off[2] = {0, 0};
  int64_t sub_off[2][8] = {};  // long lists and tiles, relative to part_off
  double nb_inf = 0.0, nc_inf = 0.0, kkt_zero = 0.0;
};

// exact symmetry of a host CSR given by pointers (dense: direct index check)
bool symmetric_ptrs(const int64_t* rowptr, const int32_t* col, const double* val, int64_t n, bool dense) {
  if (dense) {
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = i + 1; j < n; ++j)
        if (memcmp(&val[i * n + j], &val[j * n + i], sizeof(double)) != 0) return false;
    return true;
  }
  HostCsr H;
  H.nrows = H.ncols = n;
  H.rowptr.assign(rowptr, rowptr + n + 1);
  H.col.assign(col, col + rowptr[n]);
  H.val.assign(val, val + rowptr[n]);
  return exactly_symmetric(H);
}

bool is_dense(const int64_t* rowptr, int64_t n) {
  if (rowptr[n] != n * n) return false;
  for (int64_t i = 0; i <= n; ++i)
    if (rowptr[i] != i * n) return false;
  return true;
}

// Row partitions of one workgroup covering all rows, packed as: for each of
// the n-side, CG, A and A' partitions six ints (bounds[0..1], long_ptr[0..1],
// tile_ptr[0..1], the last two relative), then the four long-row lists, then
// the four tile arrays.
// workgroup sizes of the batched kernel: the default, and the alternative the
// autotuner may pick (index 1 of BatchInst's partitions)
constexpr int kBatchSizes[2] = {kBatchBlock, kSolveBlock};

void batch_parts(const int64_t* qrp, bool dense, int64_t n, const HostCsr& A, const HostCsr& T, int block,
                 std::vector<int32_t>& out, int32_t g[4], int64_t off[8]) {
  const int64_t m = A.nrows;
  const int64_t* q = dense ? nullptr : qrp;
  const int64_t* arp = m ? A.rowptr.data() : nullptr;
  const int64_t* trp = m ? T.rowptr.data() : nullptr;
  HostPart p1 = build_part(n, 1, q, trp, 0, block);
  HostPart p2 = build_part(n, 1, q, nullptr, 0, block);
  HostPart p3 = build_part(m, 1, arp, nullptr, 0, block);
  HostPart p4 = build_part(n, 1, trp, nullptr, 0, block);
  const HostPart* ps[4] = {&p1, &p2, &p3, &p4};
  const int64_t base = (int64_t)out.size();
  for (int k = 0; k < 4; ++k) {
    out.push_back(ps[k]->bounds[0]);
    out.push_back(ps[k]->bounds[1]);
    out.push_back(0);
    out.push_back((int32_t)ps[k]->long_rows.size());
    out.push_back(0);
    out.push_back(ps[k]->tile_ptr[1]);
    g[k] = ps[k]->group;
  }
  for (int k = 0; k < 4; ++k) {
    off[k] = (int64_t)out.size() - base;
    out.insert(out.end(), ps[k]->long_rows.begin(), ps[k]->long_rows.end());
  }
  for (int k = 0; k < 4; ++k) {
    off[4 + k] = (int64_t)out.size() - base;
    out.insert(out.end(), ps[k]->tiles.begin(), ps[k]->tiles.end());
  }
  if (dense) g[0] = pow2_ceil(m ? (double)T.rowptr[n] / (double)n : 1.0);
}

// Device buffers of a batch: allocated with hipMalloc (and freed with the
// batch), or, with an arena, carved from that region (the static scratch of
// the allocation-free entry point: nothing is allocated or freed).
struct DevBuf {
  std::vector<void*> ptrs;
  char* arena = nullptr;
  size_t cap = 0, used = 0;
  ~DevBuf() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <typename T>
  int alloc(T** p, int64_t count) {
    *p = nullptr;
    const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    if (arena) {
      const size_t off = (used + 255) & ~(size_t)255;
      if (off + bytes > cap)
        return fail(PDHCG_ERR_INVALID_ARGUMENT,
                    "the batch needs more device memory than the " + std::to_string(cap >> 20) +
                        " MiB static scratch of pdhcg_solve_batch_noalloc holds (at least " +
                        std::to_string(off + bytes) + " bytes); use pdhcg_solve_batch");
      *p = (T*)(arena + off);
      used = off + bytes;
      return 0;
    }
    const hipError_t e = hipMalloc((void**)p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(PDHCG_ERR_OUT_OF_MEMORY,
                  "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    ptrs.push_back(*p);
    return 0;
  }
};

}  // namespace

// A batch packed on the device once and solved any number of times: the
// matrices, vectors, row partitions, parameter blocks and (with
// preconditioning) the scaled data and D1, D2 stay resident in HBM.
struct pdhcg_batch {
  int32_t count = 0;
  hipStream_t stream = nullptr;
  pdhcg_settings s{};
  bool pre = false, mixed = false;
  int32_t nsizes = 1;                // workgroup sizes with partitions built (2: the autotuner may switch)
  int32_t threads = kBatchBlock;     // threads per workgroup of the batched kernel
  DevBuf D;
  std::vector<BatchInst> inst;
  std::vector<int64_t> off_n, off_m;  // count + 1 offsets of the packed vectors
  int64_t vn_tot = 0, vm_tot = 0;
  std::vector<int32_t> given0;        // start flags of the last solve (bit 0 x0, bit 1 y0)
  SolveParams* d_params = nullptr;
  int32_t* d_order = nullptr;
  SolverState* d_st = nullptr;
  uint64_t* d_t0 = nullptr;
  uint8_t* d_given = nullptr;
  double *d_x0 = nullptr, *d_y0 = nullptr, *d_d2 = nullptr, *d_d1 = nullptr;
  double *x = nullptr, *y = nullptr;    // packed iterates (of the scaled problems when preconditioned)
  double *xo = nullptr, *yo = nullptr;  // returned points of the callers' problems
  BatchParams bp{};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double setup_s = 0.0;
  ~pdhcg_batch() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

namespace {

// One instance's input as host arrays: the caller's own, or copies of
// device-resident input fetched once.
struct HostInst {
  pdhcg_csr Q{}, A{};
  pdhcg_lowrank L{};
  const double* b = nullptr;
  const double* c = nullptr;
  std::vector<int64_t> qrp, arp;
  std::vector<int32_t> qcol, acol;
  std::vector<double> qval, aval, bv, cv, F, d;
};

int fetch_dev(void* dst, const void* src, size_t bytes) {
  if (bytes) HIPX(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
  return 0;
}

// host copies of a CSR given in device memory (sizes are checked by the caller)
int host_csr(const pdhcg_csr& M, std::vector<int64_t>& rp, std::vector<int32_t>& col, std::vector<double>& val,
             pdhcg_csr& out) {
  out = M;
  if (!M.on_device) return 0;
  if (!M.rowptr || (M.nnz > 0 && (!M.col || !M.val))) return 0;  // reported as null arrays later
  int rc;
  rp.resize(M.nrows + 1);
  col.resize(M.nnz);
  val.resize(M.nnz);
  if ((rc = fetch_dev(rp.data(), M.rowptr, sizeof(int64_t) * (M.nrows + 1)))) return rc;
  if ((rc = fetch_dev(col.data(), M.col, sizeof(int32_t) * M.nnz))) return rc;
  if ((rc = fetch_dev(val.data(), M.val, sizeof(double) * M.nnz))) return rc;
  out.rowptr = rp.data();
  out.col = col.data();
  out.val = val.data();
  out.on_device = 0;
  return 0;
}

}  // namespace

// Pack and upload a batch; Q of instance i is Qs[i] (CSR, dense detected) or,
// when Ls is given instead, the factor Ls[i] of Q = F F' + diag(d).
int batch_create_impl(pdhcg_batch** out, int32_t count, const pdhcg_csr* Qs_in, const pdhcg_lowrank* Ls_in,
                      const pdhcg_csr* As_in, const double* const* bs_in, const double* const* cs_in,
                      int32_t vec_on_device, const pdhcg_settings* s, void* hip_stream, bool tunable,
                      char* arena = nullptr, size_t arena_bytes = 0) {
  const double t0 = now_s();
  int rc;
  if (!out) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle pointer");
  *out = nullptr;
  if ((rc = check_settings(s))) return rc;
  if (count < 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "count must be >= 1");
  if ((!Qs_in && !Ls_in) || (Qs_in && Ls_in) || !As_in || !bs_in || !cs_in)
    return fail(PDHCG_ERR_INVALID_ARGUMENT, "null array argument (exactly one of Qs and Ls must be given)");
  const bool lowrank = Ls_in != nullptr;
  // preconditioning (Sec. 4, preprocessing) per instance: every instance gets
  // its own blocks (no sharing), scaled on the device after the upload by one
  // launch (one workgroup per instance); a dense Q keeps its dense block and a
  // factored Q its factor form
  const bool pre = s->ruiz_iters != 0 || s->pock_chambolle != 0;
  const bool mixed = s->precision == 1;

  // ---- host views of the inputs (device-resident inputs are fetched once)
  std::vector<HostInst> H(count);
  for (int i = 0; i < count; ++i) {
    HostInst& hi = H[i];
    const std::string tag = "instance " + std::to_string(i);
    if ((rc = host_csr(As_in[i], hi.arp, hi.acol, hi.aval, hi.A))) return rc;
    if (lowrank) {
      hi.L = Ls_in[i];
      const pdhcg_lowrank& L = Ls_in[i];
      if (L.n < 1 || L.k < 1 || L.k > L.n || L.n >= (1 << 30) || L.n * L.k >= (1ll << 31))
        return fail(PDHCG_ERR_INVALID_ARGUMENT, tag + ": factor sizes must satisfy 1 <= k <= n < 2^30");
      if (!L.F || !L.d) return fail(PDHCG_ERR_INVALID_ARGUMENT, tag + ": null factor array");
      if (L.on_device) {
        hi.F.resize((size_t)(L.n * L.k));
        hi.d.resize((size_t)L.n);
        if ((rc = fetch_dev(hi.F.data(), L.F, sizeof(double) * hi.F.size()))) return rc;
        if ((rc = fetch_dev(hi.d.data(), L.d, sizeof(double) * hi.d.size()))) return rc;
        hi.L.F = hi.F.data();
        hi.L.d = hi.d.data();
        hi.L.on_device = 0;
      }
    } else {
      if ((rc = host_csr(Qs_in[i], hi.qrp, hi.qcol, hi.qval, hi.Q))) return rc;
    }
    const int64_t n = lowrank ? Ls_in[i].n : Qs_in[i].nrows;
    const int64_t m = As_in[i].nrows;
    if (n < 1 || n >= (1 << 30) || m < 0 || m >= (1 << 30))
      return fail(PDHCG_ERR_INVALID_ARGUMENT, tag + ": bad shapes");
    hi.b = bs_in[i];
    hi.c = cs_in[i];
    if (!hi.c || (m > 0 && !hi.b)) return fail(PDHCG_ERR_INVALID_ARGUMENT, tag + ": null array");
    if (vec_on_device) {
      hi.cv.resize(n);
      hi.bv.resize(std::max<int64_t>(m, 1), 0.0);
      if ((rc = fetch_dev(hi.cv.data(), hi.c, sizeof(double) * n))) return rc;
      if (m > 0 && (rc = fetch_dev(hi.bv.data(), hi.b, sizeof(double) * m))) return rc;
      hi.c = hi.cv.data();
      hi.b = hi.bv.data();
    }
  }
  std::vector<pdhcg_csr> Qv(count), Av(count);
  std::vector<pdhcg_lowrank> Lv(lowrank ? count : 0);
  std::vector<const double*> bs(count), cs(count);
  for (int i = 0; i < count; ++i) {
    Qv[i] = H[i].Q;
    Av[i] = H[i].A;
    if (lowrank) Lv[i] = H[i].L;
    bs[i] = H[i].b;
    cs[i] = H[i].c;
  }
  const pdhcg_csr* Qs = lowrank ? nullptr : Qv.data();
  const pdhcg_lowrank* Ls = lowrank ? Lv.data() : nullptr;
  const pdhcg_csr* As = Av.data();
  hipStream_t stream = (hipStream_t)hip_stream;

  pdhcg_batch* h = new pdhcg_batch();
  auto bail = [&](int code) {
    delete h;
    return code;
  };
  h->count = count;
  const int nsizes = tunable ? 2 : 1;  // partitions and parameter blocks for both workgroup sizes
  h->nsizes = nsizes;
  h->stream = stream;
  h->s = *s;
  h->pre = pre;
  h->mixed = mixed;
  h->D.arena = arena;
  h->D.cap = arena_bytes;

  // ---- validate, detect dense Q, build A', de-duplicate shared matrices
  std::vector<BatchInst>& inst = h->inst;
  inst.resize(count);
  std::vector<HostCsr> At(count);
  std::vector<int32_t> parts;
  struct Key {
    const void *a, *b, *c;
    bool operator<(const Key& o) const { return std::tie(a, b, c) < std::tie(o.a, o.b, o.c); }
  };
  std::map<Key, int> q_seen, a_seen;
  std::vector<int> q_first(count, -1), a_first(count, -1);
  int64_t rp_tot = 0, nz_tot = 0, vn_tot = 0, vm_tot = 0;
  for (int i = 0; i < count; ++i) {
    // a factored Q stands in as a dense n x n CSR header for the shape checks
    pdhcg_csr Qf{};
    if (Ls) {
      const pdhcg_lowrank& L = Ls[i];
      Qf.nrows = Qf.ncols = L.n;
      Qf.nnz = 2 * L.n * L.k + L.n;  // stored values: F, F', d
      Qf.rowptr = reinterpret_cast<const int64_t*>(L.F);  // (identity of the factor for sharing; not read)
      Qf.col = reinterpret_cast<const int32_t*>(L.d);
      Qf.val = L.F;
    }
    const pdhcg_csr& Q = Ls ? Qf : Qs[i];
    const pdhcg_csr& A = As[i];
    const std::string tag = "instance " + std::to_string(i);
    if (Q.nrows != Q.ncols || Q.nrows < 1 || A.ncols != Q.nrows || A.nrows < 0)
      return bail(fail(PDHCG_ERR_INVALID_ARGUMENT, tag + ": bad shapes"));
    if (Q.nrows >= (1 << 30) || A.nrows >= (1 << 30) || Q.nnz >= (1ll << 31) || A.nnz >= (1ll << 31) ||
        Q.nnz < 0 || A.nnz < 0)
      return bail(fail(PDHCG_ERR_INVALID_ARGUMENT, tag + ": sizes beyond 32-bit indexing"));
    if (!Q.rowptr || !A.rowptr || (Q.nnz && (!Q.col || !Q.val)) || (A.nnz && (!A.col || !A.val)))
      return bail(fail(PDHCG_ERR_INVALID_ARGUMENT, tag + ": null array"));
    BatchInst& I = inst[i];
    I.n = (int32_t)Q.nrows;
    I.m = (int32_t)A.nrows;
    const Key qk{Q.rowptr, Q.col, Q.val}, ak{A.rowptr, A.col, A.val};
    auto qit = pre ? q_seen.end() : q_seen.find(qk);
    if (qit == q_seen.end() && Ls) {
      I.dense = 2;
      I.q_rank = (int32_t)Ls[i].k;
      I.q_rp = 0;
      I.q_nz = nz_tot;
      nz_tot += Q.nnz;
      q_seen[qk] = i;
      q_first[i] = i;
    } else if (qit == q_seen.end()) {
      if ((rc = check_structure(Q.rowptr, Q.col, Q.nrows, Q.ncols, Q.nnz, tag + " Q"))) return bail(rc);
      const bool dense = is_dense(Q.rowptr, Q.nrows);
      if (!symmetric_ptrs(Q.rowptr, Q.col, Q.val, Q.nrows, dense))
        return bail(fail(PDHCG_ERR_INVALID_ARGUMENT, tag + ": Q is not exactly symmetric"));
      I.dense = dense ? 1 : 0;
      I.q_rp = dense ? 0 : rp_tot;
      I.q_nz = nz_tot;
      if (!dense) rp_tot += Q.nrows + 1;
      nz_tot += Q.nnz;
      q_seen[qk] = i;
      q_first[i] = i;
    } else {
      const BatchInst& F = inst[qit->second];
      I.dense = F.dense; I.q_rank = F.q_rank; I.q_rp = F.q_rp; I.q_nz = F.q_nz;
      q_first[i] = qit->second;
    }
    auto ait = pre ? a_seen.end() : a_seen.find(ak);
    if (ait == a_seen.end()) {
      if ((rc = check_structure(A.rowptr, A.col, A.nrows, A.ncols, A.nnz, tag + " A"))) return bail(rc);
      HostCsr Ah;
      Ah.nrows = A.nrows;
      Ah.ncols = A.ncols;
      Ah.rowptr.assign(A.rowptr, A.rowptr + A.nrows + 1);
      Ah.col.assign(A.col, A.col + A.nnz);
      Ah.val.assign(A.val, A.val + A.nnz);
      At[i] = transpose(Ah);
      I.a_rp = rp_tot; rp_tot += A.nrows + 1;
      I.t_rp = rp_tot; rp_tot += Q.nrows + 1;
      I.a_nz = nz_tot; nz_tot += A.nnz;
      I.t_nz = nz_tot; nz_tot += A.nnz;
      a_seen[ak] = i;
      a_first[i] = i;
    } else {
      const BatchInst& F = inst[ait->second];
      I.a_rp = F.a_rp; I.t_rp = F.t_rp; I.a_nz = F.a_nz; I.t_nz = F.t_nz;
      a_first[i] = ait->second;
    }
    I.voff_n = vn_tot; vn_tot += I.n;
    I.voff_m = vm_tot; vm_tot += I.m;
    // relKKT is that of the caller's problem: norms of the unscaled b and c
    I.nc_inf = max_abs_nan(cs[i], I.n);
    I.nb_inf = max_abs_nan(bs[i], I.m);
    I.kkt_zero = kkt_at_zero(bs[i], I.m, cs[i], I.n);
  }
  h->vn_tot = vn_tot;
  h->vm_tot = vm_tot;
  h->off_n.resize(count + 1);
  h->off_m.resize(count + 1);
  for (int i = 0; i < count; ++i) {
    h->off_n[i] = inst[i].voff_n;
    h->off_m[i] = inst[i].voff_m;
  }
  h->off_n[count] = vn_tot;
  h->off_m[count] = vm_tot;
  // partitions (per distinct (Q, A) pair the lists are identical; built per instance for simplicity)
  for (int i = 0; i < count; ++i) {
    BatchInst& I = inst[i];
    const HostCsr& T = At[a_first[i]];
    HostCsr Ah;
    Ah.nrows = As[i].nrows;
    Ah.ncols = As[i].ncols;
    Ah.rowptr.assign(As[i].rowptr, As[i].rowptr + As[i].nrows + 1);
    for (int z = 0; z < nsizes; ++z) {
      I.part_off[z] = (int64_t)parts.size();
      batch_parts(Ls ? nullptr : Qs[q_first[i]].rowptr, I.dense != 0, I.n, Ah, T, kBatchSizes[z], parts, I.g[z],
                  I.sub_off[z]);
    }
  }
  // largest first: estimated work ~ entries of Q plus twice those of A
  std::vector<int32_t> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    auto qnz = [&](int i) { return Ls ? 2.0 * (double)Ls[i].n * (double)Ls[i].k : (double)Qs[i].nnz; };
    const double wa = qnz(a) + 2.0 * (double)As[a].nnz + inst[a].n;
    const double wb = qnz(b) + 2.0 * (double)As[b].nnz + inst[b].n;
    return wa > wb;
  });

  // ---- device buffers
  DevBuf& D = h->D;
  int32_t *d_rp, *d_col, *d_parts;
  double* d_val;
  float* d_val32 = nullptr;
  double *d_b, *d_c, *d_part;
  double* nv[10];  // x xa x_anc r p0 p1 q x_prev (+ F' v of a factored Q) (+ kept Q x of a dense Q)
  double* mv[7];  // y ya ax ax_avg y_anc y_trial ax_trial
  float* fv[1] = {nullptr};        // x32
  float2* d_rp32 = nullptr;        // FP32 (r, p) records of the textbook CG
  if ((rc = D.alloc(&d_rp, rp_tot))) return bail(rc);
  if ((rc = D.alloc(&d_col, nz_tot))) return bail(rc);
  if ((rc = D.alloc(&d_val, nz_tot))) return bail(rc);
  // (+4: the 16-byte loads of the dense FP32 products may read up to three
  // values past the last matrix)
  if (mixed && (rc = D.alloc(&d_val32, nz_tot + 4))) return bail(rc);
  if ((rc = D.alloc(&d_parts, (int64_t)parts.size()))) return bail(rc);
  if ((rc = D.alloc(&h->d_params, (int64_t)count * nsizes))) return bail(rc);
  if ((rc = D.alloc(&h->d_st, count))) return bail(rc);
  if ((rc = D.alloc(&h->d_t0, 1))) return bail(rc);
  if ((rc = D.alloc(&h->d_given, count))) return bail(rc);
  if ((rc = D.alloc(&d_b, vm_tot))) return bail(rc);
  if ((rc = D.alloc(&d_c, vn_tot))) return bail(rc);
  if ((rc = D.alloc(&d_part, (int64_t)count * NSLOT))) return bail(rc);
  if ((rc = D.alloc(&h->d_order, count))) return bail(rc);
  const bool adaptive = s->step_rule == 1;
  bool any_dense = false;
  for (int i = 0; i < count; ++i) any_dense |= inst[i].dense != 0;
  for (int k = 0; k < 10; ++k) {
    nv[k] = nullptr;
    if ((k == 7 && !adaptive) || (k == 8 && !Ls) || (k == 9 && (adaptive || !any_dense))) continue;
    if ((rc = D.alloc(&nv[k], vn_tot))) return bail(rc);
  }
  for (int k = 0; k < 7; ++k) {
    mv[k] = nullptr;
    if (k >= 5 && !adaptive) continue;
    if ((rc = D.alloc(&mv[k], vm_tot))) return bail(rc);
  }
  if (mixed && ((rc = D.alloc(&fv[0], vn_tot)) || (rc = D.alloc(&d_rp32, vn_tot)))) return bail(rc);
  if ((rc = D.alloc(&h->d_x0, vn_tot))) return bail(rc);
  if ((rc = D.alloc(&h->d_y0, vm_tot))) return bail(rc);
  if ((rc = D.alloc(&h->xo, vn_tot))) return bail(rc);
  if ((rc = D.alloc(&h->yo, vm_tot))) return bail(rc);
  h->x = nv[0];
  h->y = mv[0];

  // ---- uploads (matrix blocks straight from the host arrays)
  auto up = [&](void* dst, const void* src, size_t bytes) -> int {
    if (bytes) HIPX(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream));
    return 0;
  };
  std::vector<std::vector<int32_t>> rp_keep;
  std::vector<std::vector<double>> val_keep;  // factor blocks, alive until the uploads complete
  for (int i = 0; i < count; ++i) {
    const BatchInst& I = inst[i];
    if (q_first[i] == i && Ls) {  // block [F (n x k) | F' (k x n) | d (n)], row-major
      const pdhcg_lowrank& L = Ls[i];
      const int64_t n = L.n, k = L.k;
      std::vector<double> blk((size_t)(2 * n * k + n));
      memcpy(blk.data(), L.F, sizeof(double) * (size_t)(n * k));
      for (int64_t r = 0; r < n; ++r)
        for (int64_t c = 0; c < k; ++c) blk[(size_t)(n * k + c * n + r)] = L.F[r * k + c];
      memcpy(blk.data() + 2 * n * k, L.d, sizeof(double) * (size_t)n);
      val_keep.push_back(std::move(blk));
      if ((rc = up(d_val + I.q_nz, val_keep.back().data(), sizeof(double) * val_keep.back().size()))) return bail(rc);
    } else if (q_first[i] == i) {
      const pdhcg_csr& Q = Qs[i];
      if (!I.dense) {
        rp_keep.emplace_back(Q.rowptr, Q.rowptr + Q.nrows + 1);
        if ((rc = up(d_rp + I.q_rp, rp_keep.back().data(), sizeof(int32_t) * (Q.nrows + 1)))) return bail(rc);
        if ((rc = up(d_col + I.q_nz, Q.col, sizeof(int32_t) * Q.nnz))) return bail(rc);
      }
      if ((rc = up(d_val + I.q_nz, Q.val, sizeof(double) * Q.nnz))) return bail(rc);
    }
    if (a_first[i] == i) {
      const pdhcg_csr& A = As[i];
      const HostCsr& T = At[i];
      rp_keep.emplace_back(A.rowptr, A.rowptr + A.nrows + 1);
      if ((rc = up(d_rp + I.a_rp, rp_keep.back().data(), sizeof(int32_t) * (A.nrows + 1)))) return bail(rc);
      rp_keep.emplace_back(T.rowptr.begin(), T.rowptr.end());
      if ((rc = up(d_rp + I.t_rp, rp_keep.back().data(), sizeof(int32_t) * (T.nrows + 1)))) return bail(rc);
      if ((rc = up(d_col + I.a_nz, A.col, sizeof(int32_t) * A.nnz))) return bail(rc);
      if ((rc = up(d_val + I.a_nz, A.val, sizeof(double) * A.nnz))) return bail(rc);
      if ((rc = up(d_col + I.t_nz, T.col.data(), sizeof(int32_t) * A.nnz))) return bail(rc);
      if ((rc = up(d_val + I.t_nz, T.val.data(), sizeof(double) * A.nnz))) return bail(rc);
    }
    if ((rc = up(d_c + I.voff_n, cs[i], sizeof(double) * I.n))) return bail(rc);
    if (I.m && (rc = up(d_b + I.voff_m, bs[i], sizeof(double) * I.m))) return bail(rc);
  }
  // ---- preconditioning: one launch scales every instance's blocks; D2 packed
  // like x, D1 like y; b and c scaled in place
  if (pre) {
    double* d_f = nullptr;
    PrecInst* d_pi = nullptr;
    if ((rc = D.alloc(&d_f, vn_tot + vm_tot))) return bail(rc);
    if ((rc = D.alloc(&h->d_d2, vn_tot))) return bail(rc);
    if ((rc = D.alloc(&h->d_d1, std::max<int64_t>(vm_tot, 1)))) return bail(rc);
    if ((rc = D.alloc(&d_pi, count))) return bail(rc);
    const std::vector<double> ones((size_t)std::max(vn_tot, vm_tot), 1.0);
    if ((rc = up(h->d_d2, ones.data(), sizeof(double) * vn_tot))) return bail(rc);
    if ((rc = up(h->d_d1, ones.data(), sizeof(double) * vm_tot))) return bail(rc);
    std::vector<PrecInst> pi(count);
    for (int i = 0; i < count; ++i) {
      const BatchInst& I = inst[i];
      PrecInst& P = pi[i];
      P.n = I.n;
      P.m = I.m;
      P.qkind = I.dense;
      P.k = I.q_rank;
      P.qrp = I.dense ? nullptr : d_rp + I.q_rp;
      P.qcol = I.dense ? nullptr : d_col + I.q_nz;
      P.qval = d_val + I.q_nz;
      P.arp = d_rp + I.a_rp;
      P.acol = d_col + I.a_nz;
      P.aval = d_val + I.a_nz;
      P.trp = d_rp + I.t_rp;
      P.tcol = d_col + I.t_nz;
      P.tval = d_val + I.t_nz;
      P.d2 = h->d_d2 + I.voff_n;
      P.d1 = h->d_d1 + I.voff_m;
      P.f = d_f + I.voff_n + I.voff_m;
      const int64_t nnzq = I.dense ? 0 : Qs[i].nnz;
      P.gk = precond_lanes(nnzq + 2 * As[i].nnz, (int64_t)I.n + I.m);
      P.gq = precond_lanes(nnzq, I.n);
      P.ga = precond_lanes(As[i].nnz, I.m);
      P.gt = precond_lanes(As[i].nnz, I.n);
    }
    if ((rc = up(d_pi, pi.data(), sizeof(PrecInst) * count))) return bail(rc);
    if (launch_batch_precondition(d_pi, count, s->ruiz_iters, s->pock_chambolle, stream) != hipSuccess ||
        launch_diag(d_c, h->d_d2, vn_tot, 0, d_c, stream) != hipSuccess ||
        launch_diag(d_b, h->d_d1, vm_tot, 0, d_b, stream) != hipSuccess)
      return bail(fail(PDHCG_ERR_HIP, "preconditioning kernels failed to launch"));
  }
  // one parameter block per QP, all pointers resolved against the packed arrays
  std::vector<SolveParams> hp((size_t)count * nsizes);
  for (int i = 0; i < count; ++i) {
    const BatchInst& I = inst[i];
    SolveParams& P = hp[i];
    P.Q = DevMat{I.n, I.n, I.dense ? nullptr : d_rp + I.q_rp, I.dense ? nullptr : d_col + I.q_nz, d_val + I.q_nz,
                 d_val32 ? d_val32 + I.q_nz : nullptr, I.dense, I.q_rank};
    P.lr_t = Ls ? nv[8] + I.voff_n : nullptr;
    P.A = DevMat{I.m, I.n, d_rp + I.a_rp, d_col + I.a_nz, d_val + I.a_nz, d_val32 ? d_val32 + I.a_nz : nullptr, 0};
    P.At = DevMat{I.n, I.m, d_rp + I.t_rp, d_col + I.t_nz, d_val + I.t_nz, d_val32 ? d_val32 + I.t_nz : nullptr, 0};
    P.n = I.n;
    P.m = I.m;
    P.b = d_b + I.voff_m;
    P.c = d_c + I.voff_n;
    P.x = nv[0] + I.voff_n; P.xa = nv[1] + I.voff_n; P.x_anc = nv[2] + I.voff_n; P.r = nv[3] + I.voff_n;
    P.p0 = nv[4] + I.voff_n; P.p1 = nv[5] + I.voff_n; P.q = nv[6] + I.voff_n;
    P.y = mv[0] + I.voff_m; P.ya = mv[1] + I.voff_m; P.ax = mv[2] + I.voff_m; P.ax_avg = mv[3] + I.voff_m;
    P.y_anc = mv[4] + I.voff_m;
    if (mixed) {
      P.x32 = fv[0] + I.voff_n; P.rp32 = d_rp32 + I.voff_n;
    }
    P.part = d_part + (int64_t)i * NSLOT;
    const int32_t* pb = d_parts + I.part_off[0];
    auto part = [&](int k) {
      return Part{pb + 6 * k, pb + 6 * k + 2, pb + I.sub_off[0][k], pb + 6 * k + 4, pb + I.sub_off[0][4 + k],
                  I.g[0][k]};
    };
    P.pn1 = part(0);
    P.pcg = part(1);
    P.pm = part(2);
    P.pt = part(3);
    P.nb_inf = I.nb_inf;
    P.nc_inf = I.nc_inf;
    P.dn = pre ? h->d_d2 + I.voff_n : nullptr;
    P.dm = pre && I.m > 0 ? h->d_d1 + I.voff_m : nullptr;
    P.kkt_zero = I.kkt_zero;  // (applied only to a given start, per solve)
    P.x0 = h->d_x0 + I.voff_n;
    P.y0 = h->d_y0 + I.voff_m;
    P.tol = s->tol_rel_kkt; P.eps_factor = s->cg_eps_factor; P.beta_suf = s->beta_sufficient;
    P.beta_nec = s->beta_necessary; P.beta_art = s->beta_artificial; P.theta = s->primal_weight_theta;
    P.max_iters = s->max_iters;
    P.iters_this_launch = s->max_iters;
    P.time_limit_ticks = s->time_limit_s > 0.0 ? (uint64_t)(s->time_limit_s * 1e8) : 0;
    P.max_cg = s->max_cg_iters; P.cg_rule = s->cg_rule; P.restart_to = s->restart_to;
    P.eval_period = s->eval_period;
    P.mixed_allowed = mixed ? 1 : 0;
    P.step_rule = s->step_rule;
    if (I.dense && nv[9]) P.qx = nv[9] + I.voff_n;
    if (adaptive) {
      P.x_prev = nv[7] + I.voff_n;
      P.y_trial = mv[5] + I.voff_m;
      P.ax_trial = mv[6] + I.voff_m;
    }
  }
  if ((rc = up(d_parts, parts.data(), sizeof(int32_t) * parts.size()))) return bail(rc);
  if ((rc = up(h->d_order, order.data(), sizeof(int32_t) * count))) return bail(rc);
  for (int z = 1; z < nsizes; ++z)  // the same blocks with the partitions cut for the other workgroup size
    for (int i = 0; i < count; ++i) {
      const BatchInst& I = inst[i];
      SolveParams& P = hp[(size_t)z * count + i];
      P = hp[i];
      const int32_t* pb = d_parts + I.part_off[z];
      auto part = [&](int k) {
        return Part{pb + 6 * k, pb + 6 * k + 2, pb + I.sub_off[z][k], pb + 6 * k + 4, pb + I.sub_off[z][4 + k],
                    I.g[z][k]};
      };
      P.pn1 = part(0);
      P.pcg = part(1);
      P.pm = part(2);
      P.pt = part(3);
    }
  if ((rc = up(h->d_params, hp.data(), sizeof(SolveParams) * hp.size()))) return bail(rc);
  if (mixed && launch_to_f32(d_val, d_val32, nz_tot, stream) != hipSuccess)
    return bail(fail(PDHCG_ERR_HIP, "FP32 conversion failed to launch"));
  if (hipStreamSynchronize(stream) != hipSuccess) return bail(fail(PDHCG_ERR_HIP, "batch upload or setup failed"));
  rp_keep.clear();
  // (without events in the allocation-free form: its solve time is host wall time)
  if (!arena && (hipEventCreate(&h->e0) != hipSuccess || hipEventCreate(&h->e1) != hipSuccess))
    return bail(fail(PDHCG_ERR_HIP, "hipEventCreate failed"));

  BatchParams& bp = h->bp;
  bp.params = h->d_params;
  bp.order = h->d_order;
  bp.st = h->d_st;
  bp.t0 = h->d_t0;
  bp.pw_init = s->primal_weight_init;
  bp.eta_factor = s->step_eta_factor;
  bp.power_iters = s->power_iters;
  bp.mixed = mixed ? 1 : 0;
  bp.given = h->d_given;
  bp.warm_fallback = s->warm_fallback;
  h->setup_s = now_s() - t0;
  *out = h;
  return 0;
}

namespace {

// The batch's start stamp and its one launch at the handle's workgroup size
// (the parameter blocks of that size's partitions)
hipError_t launch_batch(pdhcg_batch* h, hipStream_t stream) {
  BatchParams bp = h->bp;
  const int z = h->threads == kBatchSizes[1] ? 1 : 0;
  bp.params = h->d_params + (size_t)z * h->count;
  hipError_t e = launch_batch_clock(bp.t0, stream);
  if (e != hipSuccess) return e;
  return z ? launch_batch_512(bp, h->count, stream) : launch_batch_256(bp, h->count, stream);
}

// Solve every instance of a packed batch.  x0 / y0: packed start points
// (device pointers when in_dev; may be null) with per-instance flags in
// `given` (bit 0 x0, bit 1 y0; null: every instance takes the given vectors);
// x_out / y_out: packed outputs (device pointers when out_dev).
int batch_solve_impl(pdhcg_batch* h, const double* x0, const double* y0, bool in_dev, const uint8_t* given,
                     double* x_out, double* y_out, bool out_dev, pdhcg_result* rs) {
  const double t0 = now_s();
  hipStream_t stream = h->stream;
  const int count = h->count;
  const hipMemcpyKind in_kind = in_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  std::vector<uint8_t> g(count, 0);
  for (int i = 0; i < count; ++i) {
    const bool has_m = h->inst[i].m > 0;
    g[i] = given ? (uint8_t)(given[i] & (has_m ? 3 : 1)) : (uint8_t)((x0 ? 1 : 0) | (y0 && has_m ? 2 : 0));
  }
  if (x0) HIPX(hipMemcpyAsync(h->d_x0, x0, sizeof(double) * h->vn_tot, in_kind, stream));
  if (y0 && h->vm_tot) HIPX(hipMemcpyAsync(h->d_y0, y0, sizeof(double) * h->vm_tot, in_kind, stream));
  if (h->pre) {  // x~ = x / D2, y~ = y / D1
    if (x0) HIPX(launch_diag(h->d_x0, h->d_d2, h->vn_tot, 1, h->d_x0, stream));
    if (y0) HIPX(launch_diag(h->d_y0, h->d_d1, h->vm_tot, 1, h->d_y0, stream));
  }
  HIPX(hipMemcpyAsync(h->d_given, g.data(), (size_t)count, hipMemcpyHostToDevice, stream));
  if (h->e0) HIPX(hipEventRecord(h->e0, stream));
  HIPX(launch_batch(h, stream));
  if (h->e1) HIPX(hipEventRecord(h->e1, stream));
  const double* xr = h->x;
  const double* yr = h->y;
  if (h->pre) {  // x = D2 x~, y = D1 y~
    HIPX(launch_diag(h->x, h->d_d2, h->vn_tot, 0, h->xo, stream));
    HIPX(launch_diag(h->y, h->d_d1, h->vm_tot, 0, h->yo, stream));
    xr = h->xo;
    yr = h->yo;
  }
  const hipMemcpyKind out_kind = out_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  std::vector<SolverState> st(count);
  HIPX(hipMemcpyAsync(st.data(), h->d_st, sizeof(SolverState) * count, hipMemcpyDeviceToHost, stream));
  HIPX(hipMemcpyAsync(x_out, xr, sizeof(double) * h->vn_tot, out_kind, stream));
  if (h->vm_tot) HIPX(hipMemcpyAsync(y_out, yr, sizeof(double) * h->vm_tot, out_kind, stream));
  HIPX(hipStreamSynchronize(stream));
  const double t_solve = now_s() - t0;
  float ms = (float)(t_solve * 1e3);
  if (h->e0) HIPX(hipEventElapsedTime(&ms, h->e0, h->e1));
  for (int i = 0; i < count; ++i) {
    if (!rs) break;
    const SolverState& S = st[i];
    pdhcg_result& r = rs[i];
    r.status = S.status;
    r.returned_average = S.returned_average;
    r.rel_primal = S.r_p; r.rel_dual = S.r_d; r.rel_gap = S.r_g; r.rel_kkt = S.kkt;
    r.primal_obj = S.pobj; r.dual_obj = S.dobj;
    r.iters = S.k_total; r.cg_iters_total = S.cg_total; r.restarts = S.restarts;
    r.norm_A = S.norm_A;
    r.setup_s = h->setup_s;
    r.solve_s = t_solve;
    r.kernel_s = ms * 1e-3;
    r.kkt_evals = S.evals;
    r.cold_fallback = S.cold_fallback;
    r.rejected_steps = S.rejections;
    r.qx_formed = S.qx_formed;
    r.step_eta = S.eta;
  }
  return 0;
}

// The one-call batched entry points: create, solve from per-instance start
// points (null entries: cold), unpack, destroy.
int solve_batch_once(int32_t count, const pdhcg_csr* Qs, const pdhcg_lowrank* Ls, const pdhcg_csr* As,
                     const double* const* bs, const double* const* cs, const double* const* x0s,
                     const double* const* y0s, double* const* x_outs, double* const* y_outs, pdhcg_result* rs,
                     const pdhcg_settings* s, void* hip_stream, char* arena = nullptr, size_t arena_bytes = 0) {
  if (count < 0) return fail(PDHCG_ERR_INVALID_ARGUMENT, "count must be >= 0");
  if (count == 0) return 0;
  if (!x_outs || !y_outs) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null array argument");
  for (int i = 0; i < count; ++i) {
    const int64_t m = As ? As[i].nrows : 0;
    if (!x_outs[i] || (m > 0 && !y_outs[i]))
      return fail(PDHCG_ERR_INVALID_ARGUMENT, "instance " + std::to_string(i) + ": null array");
  }
  pdhcg_batch* h = nullptr;
  int rc = batch_create_impl(&h, count, Qs, Ls, As, bs, cs, 0, s, hip_stream, false, arena, arena_bytes);
  if (rc) return rc;
  std::vector<double> X0, Y0, X((size_t)h->vn_tot), Y((size_t)std::max<int64_t>(h->vm_tot, 1));
  std::vector<uint8_t> given(count, 0);
  bool any = false;
  for (int i = 0; i < count; ++i) {
    const bool gx = x0s && x0s[i], gy = y0s && y0s[i] && h->inst[i].m > 0;
    given[i] = (uint8_t)((gx ? 1 : 0) | (gy ? 2 : 0));
    any |= gx || gy;
  }
  if (any) {
    X0.assign((size_t)h->vn_tot, 0.0);
    Y0.assign((size_t)std::max<int64_t>(h->vm_tot, 1), 0.0);
    for (int i = 0; i < count; ++i) {
      const BatchInst& I = h->inst[i];
      if (given[i] & 1) memcpy(X0.data() + I.voff_n, x0s[i], sizeof(double) * I.n);
      if (given[i] & 2) memcpy(Y0.data() + I.voff_m, y0s[i], sizeof(double) * I.m);
    }
  }
  rc = batch_solve_impl(h, any ? X0.data() : nullptr, any ? Y0.data() : nullptr, false, given.data(), X.data(),
                        Y.data(), false, rs);
  if (rc == 0)
    for (int i = 0; i < count; ++i) {
      const BatchInst& I = h->inst[i];
      memcpy(x_outs[i], X.data() + I.voff_n, sizeof(double) * I.n);
      if (I.m) memcpy(y_outs[i], Y.data() + I.voff_m, sizeof(double) * I.m);
    }
  delete h;
  return rc;
}

}  // namespace

extern "C" int pdhcg_batch_create(pdhcg_batch** h, int32_t count, const pdhcg_csr* Qs, const pdhcg_lowrank* Ls,
                                  const pdhcg_csr* As, const double* const* bs, const double* const* cs,
                                  int32_t vec_on_device, const pdhcg_settings* s, void* hip_stream) {
  return batch_create_impl(h, count, Qs, Ls, As, bs, cs, vec_on_device, s, hip_stream, true);
}

extern "C" int pdhcg_batch_layout(const pdhcg_batch* h, int64_t* n_off, int64_t* m_off) {
  if (!h || !n_off || !m_off) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle or output");
  memcpy(n_off, h->off_n.data(), sizeof(int64_t) * h->off_n.size());
  memcpy(m_off, h->off_m.data(), sizeof(int64_t) * h->off_m.size());
  return 0;
}

extern "C" int pdhcg_batch_solve(pdhcg_batch* h, const double* x0, const double* y0, double* x_out, double* y_out,
                                 int32_t vec_on_device, pdhcg_result* rs) {
  if (!h) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle");
  if (!x_out || (h->vm_tot > 0 && !y_out)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null output");
  return batch_solve_impl(h, x0, y0, vec_on_device != 0, nullptr, x_out, y_out, vec_on_device != 0, rs);
}

extern "C" int pdhcg_batch_set_threads(pdhcg_batch* h, int32_t threads) {
  if (!h) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle");
  if (threads != kBatchSizes[0] && !(threads == kBatchSizes[1] && h->nsizes == 2))
    return fail(PDHCG_ERR_INVALID_ARGUMENT,
                "threads per workgroup must be 256, or 512 for a batch made by pdhcg_batch_create");
  h->threads = threads;
  return 0;
}

extern "C" int pdhcg_batch_autotune(pdhcg_batch* h, int32_t reps, int32_t* threads, double* kernel_s) {
  if (!h || !threads) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle or output");
  if (reps < 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "reps must be >= 1");
  if (h->nsizes != 2 || !h->e0) return fail(PDHCG_ERR_INVALID_ARGUMENT, "the batch was not made by pdhcg_batch_create");
  const std::vector<uint8_t> cold((size_t)h->count, 0);
  double best = INFINITY;
  int32_t pick = h->threads;
  for (int z = 0; z < 2; ++z) {
    h->threads = kBatchSizes[z];
    double tmin = INFINITY;
    for (int r = 0; r < reps; ++r) {  // a cold solve of every instance; only the launch is timed
      HIPX(hipMemcpyAsync(h->d_given, cold.data(), cold.size(), hipMemcpyHostToDevice, h->stream));
      HIPX(hipEventRecord(h->e0, h->stream));
      HIPX(launch_batch(h, h->stream));
      HIPX(hipEventRecord(h->e1, h->stream));
      HIPX(hipStreamSynchronize(h->stream));
      float ms = 0.0f;
      HIPX(hipEventElapsedTime(&ms, h->e0, h->e1));
      tmin = std::min(tmin, 1e-3 * (double)ms);
    }
    if (kernel_s) kernel_s[z] = tmin;
    if (tmin < best) {
      best = tmin;
      pick = kBatchSizes[z];
    }
  }
  h->threads = pick;
  *threads = pick;
  return 0;
}

extern "C" int pdhcg_batch_get_scaling(const pdhcg_batch* h, double* d1_out, double* d2_out, int32_t vec_on_device) {
  if (!h || !d2_out || (h->vm_tot > 0 && !d1_out)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle or output");
  const hipMemcpyKind kind = vec_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (h->pre) {
    HIPX(hipMemcpyAsync(d2_out, h->d_d2, sizeof(double) * h->vn_tot, kind, h->stream));
    if (h->vm_tot) HIPX(hipMemcpyAsync(d1_out, h->d_d1, sizeof(double) * h->vm_tot, kind, h->stream));
    HIPX(hipStreamSynchronize(h->stream));
    return 0;
  }
  const std::vector<double> ones((size_t)std::max(h->vn_tot, h->vm_tot), 1.0);
  const hipMemcpyKind hk = vec_on_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost;
  HIPX(hipMemcpy(d2_out, ones.data(), sizeof(double) * h->vn_tot, hk));
  if (h->vm_tot) HIPX(hipMemcpy(d1_out, ones.data(), sizeof(double) * h->vm_tot, hk));
  return 0;
}

extern "C" void pdhcg_batch_destroy(pdhcg_batch* h) { delete h; }

extern "C" int pdhcg_solve_batch(int32_t count, const pdhcg_csr* Qs, const pdhcg_csr* As, const double* const* bs,
                                 const double* const* cs, const double* const* x0s, const double* const* y0s,
                                 double* const* x_outs, double* const* y_outs, pdhcg_result* rs,
                                 const pdhcg_settings* s, void* hip_stream) {
  if (!Qs) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null array argument");
  return solve_batch_once(count, Qs, nullptr, As, bs, cs, x0s, y0s, x_outs, y_outs, rs, s, hip_stream);
}

int pdhcg::solve_batch_in_region(int32_t count, const pdhcg_csr* Qs, const pdhcg_csr* As, const double* const* bs,
                                 const double* const* cs, const double* const* x0s, const double* const* y0s,
                                 double* const* x_outs, double* const* y_outs, pdhcg_result* rs,
                                 const pdhcg_settings* s, void* hip_stream, char* region, size_t region_bytes) {
  if (!Qs) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null array argument");
  if (!region && count > 0) return fail(PDHCG_ERR_HIP, "no device region");
  return solve_batch_once(count, Qs, nullptr, As, bs, cs, x0s, y0s, x_outs, y_outs, rs, s, hip_stream, region,
                          region_bytes);
}

extern "C" int pdhcg_solve_batch_lowrank(int32_t count, const pdhcg_lowrank* Qs, const pdhcg_csr* As,
                                         const double* const* bs, const double* const* cs,
                                         const double* const* x0s, const double* const* y0s,
                                         double* const* x_outs, double* const* y_outs, pdhcg_result* rs,
                                         const pdhcg_settings* s, void* hip_stream) {
  if (!Qs) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null array argument");
  return solve_batch_once(count, nullptr, Qs, As, bs, cs, x0s, y0s, x_outs, y_outs, rs, s, hip_stream);
}

// One family, many right-hand sides: the batch entry point with the shared
// arrays passed for every instance (the packer stores a matrix given by the
// same host pointers once).
extern "C" int pdhcg_solve_multi_rhs(int32_t count, const pdhcg_csr* Q, const pdhcg_csr* A, const double* B,
                                     const double* c, const double* X0, const double* Y0, double* X, double* Y,
                                     pdhcg_result* rs, const pdhcg_settings* s, void* hip_stream) {
  if (count < 0) return fail(PDHCG_ERR_INVALID_ARGUMENT, "count must be >= 0");
  if (count == 0) return 0;
  if (!Q || !A || !c || !X || (A->nrows > 0 && (!B || !Y)))
    return fail(PDHCG_ERR_INVALID_ARGUMENT, "null argument");
  const int64_t n = Q->nrows, m = A->nrows;
  std::vector<pdhcg_csr> Qs(count, *Q), As(count, *A);
  std::vector<const double*> bs(count), cs(count, c), x0s(count), y0s(count);
  std::vector<double*> xs(count), ys(count);
  static double no_rows = 0.0;  // b and y of an instance without rows are never read
  for (int32_t i = 0; i < count; ++i) {
    bs[i] = m > 0 ? B + (int64_t)i * m : &no_rows;
    x0s[i] = X0 ? X0 + (int64_t)i * n : nullptr;
    y0s[i] = Y0 ? Y0 + (int64_t)i * m : nullptr;
    xs[i] = X + (int64_t)i * n;
    ys[i] = m > 0 ? Y + (int64_t)i * m : &no_rows;
  }
  return pdhcg_solve_batch(count, Qs.data(), As.data(), bs.data(), cs.data(), X0 ? x0s.data() : nullptr,
                           Y0 ? y0s.data() : nullptr, xs.data(), ys.data(), rs, s, hip_stream);
}
