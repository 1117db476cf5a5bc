// Host side of the C ABI in include/pdhcg.h: input validation, A' build,
// row-partition planning, device uploads, and the solve driver that launches
// the persistent kernel and reads back its scalar state.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <limits>
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

#define HIPX(call)                                                                         \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess) return fail(PDHCG_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
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
  if (H.rowptr[0] != 0 || H.rowptr[H.nrows] != M->nnz)
    return fail(PDHCG_ERR_INVALID_ARGUMENT, std::string(name) + ": rowptr[0] != 0 or rowptr[nrows] != nnz");
  for (int64_t i = 0; i < H.nrows; ++i) {
    if (H.rowptr[i + 1] < H.rowptr[i])
      return fail(PDHCG_ERR_INVALID_ARGUMENT, std::string(name) + ": rowptr not monotone at row " + std::to_string(i));
    for (int64_t k = H.rowptr[i]; k < H.rowptr[i + 1]; ++k) {
      if (H.col[k] < 0 || H.col[k] >= H.ncols)
        return fail(PDHCG_ERR_INVALID_ARGUMENT, std::string(name) + ": column out of range in row " + std::to_string(i));
      if (k > H.rowptr[i] && H.col[k] <= H.col[k - 1])
        return fail(PDHCG_ERR_INVALID_ARGUMENT,
                    std::string(name) + ": columns not strictly increasing in row " + std::to_string(i));
    }
  }
  return 0;
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
  std::vector<int32_t> bounds, long_ptr, long_rows;
  int32_t group = 1;
};

int pow2_ceil(double v) {
  int g = 1;
  while (g < v && g < 64) g <<= 1;
  return g;
}

// Contiguous row ranges of near-equal work (row length + 2 per row) for nb
// workgroups; rows longer than kLongRow are listed per workgroup.  The lane
// group is the power of two at or above the mean length of the other rows.
template <typename Len>
HostPart build_part(int64_t nrows, int nb, Len len) {
  HostPart P;
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
  for (int b = 0; b < nb; ++b) {
    for (int64_t i = P.bounds[b]; i < P.bounds[b + 1]; ++i)
      if (len(i) > kLongRow) P.long_rows.push_back((int32_t)i);
    P.long_ptr[b + 1] = (int32_t)P.long_rows.size();
  }
  const double mean = short_rows ? (double)short_nnz / (double)short_rows : 1.0;
  P.group = pow2_ceil(mean);
  return P;
}

}  // namespace

struct DevPart {
  int32_t* bounds = nullptr;
  int32_t* long_ptr = nullptr;
  int32_t* long_rows = nullptr;
  int32_t group = 1;
  int64_t nlong = 0;
  Part view() const { return Part{bounds, long_ptr, long_rows, group}; }
};

struct pdhcg_handle {
  int64_t n = 0, m = 0;
  int64_t nnzQ = 0, nnzA = 0;
  hipStream_t stream = nullptr;
  pdhcg_settings s{};
  int nb = 0;                 // workgroups of the persistent kernels
  int nb_spmv = 0;            // workgroups of the standalone product kernels
  double norm_A = 0.0, nb_inf = 0.0, nc_inf = 0.0, setup_s = 0.0;
  // device data
  int32_t *q_rowptr = nullptr, *q_col = nullptr, *a_rowptr = nullptr, *a_col = nullptr, *t_rowptr = nullptr,
          *t_col = nullptr;
  double *q_val = nullptr, *a_val = nullptr, *t_val = nullptr;
  float *q_val32 = nullptr, *a_val32 = nullptr, *t_val32 = nullptr;
  double *b = nullptr, *c = nullptr;
  double *x = nullptr, *y = nullptr, *xa = nullptr, *ya = nullptr, *ax = nullptr, *ax_avg = nullptr,
         *x_anc = nullptr, *y_anc = nullptr, *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
  float *x32 = nullptr, *r32 = nullptr, *p32_0 = nullptr, *p32_1 = nullptr, *xs32 = nullptr;
  double *part = nullptr, *tmp_x0 = nullptr, *tmp_y0 = nullptr, *scratch = nullptr;
  uint64_t* bar = nullptr;
  SolverState* st = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  DevPart pn1, pcg, pm, pt;                // parts for the persistent kernels
  DevPart sq, sa, st_;                     // parts for the standalone products
  std::vector<void*> allocs;

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
      return fail(PDHCG_ERR_OUT_OF_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    allocs.push_back(*p);
    return 0;
  }

  DevMat mat(int which) const {
    if (which == 0) return DevMat{(int32_t)n, (int32_t)n, q_rowptr, q_col, q_val, q_val32};
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
  if ((rc = h->alloc(&h->r32, h->n))) return rc;
  if ((rc = h->alloc(&h->p32_0, h->n))) return rc;
  if ((rc = h->alloc(&h->p32_1, h->n))) return rc;
  if ((rc = h->alloc(&h->xs32, std::max(h->n, h->m)))) return rc;
  HIPX(launch_to_f32(h->q_val, h->q_val32, h->nnzQ, h->stream));
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
  return 0;
}

int plan(pdhcg_handle* h, const HostCsr& Q, const HostCsr& A, const HostCsr& T) {
  int rc;
  int dev = 0, cus = 0;
  HIPX(hipGetDevice(&dev));
  HIPX(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  int per_cu = 0;
  HIPX(solve_occupancy(&per_cu));
  const int max_nb = std::max(1, std::min(cus * std::max(per_cu, 1), 1024));
  int nb = h->s.num_blocks;
  if (nb == 0) {
    const double work = (double)h->nnzQ + 0.25 * (double)h->nnzA + (double)(h->n + h->m);
    nb = 8;
    while (nb < 256 && work / nb > 4096.0) nb <<= 1;
  }
  nb = std::min(nb, max_nb);
  h->nb = nb;
  const HostCsr* Ap = &A;
  const HostCsr* Tp = &T;
  auto qlen = [&](int64_t i) { return Q.rowptr[i + 1] - Q.rowptr[i]; };
  auto alen = [&](int64_t i) { return Ap->nrows ? Ap->rowptr[i + 1] - Ap->rowptr[i] : 0; };
  auto tlen = [&](int64_t i) { return Ap->nrows ? Tp->rowptr[i + 1] - Tp->rowptr[i] : 0; };
  auto n1len = [&](int64_t i) { return qlen(i) + tlen(i); };
  if ((rc = upload_part(h, build_part(h->n, nb, n1len), h->pn1))) return rc;
  if ((rc = upload_part(h, build_part(h->n, nb, qlen), h->pcg))) return rc;
  if ((rc = upload_part(h, build_part(h->m, nb, alen), h->pm))) return rc;
  if ((rc = upload_part(h, build_part(h->n, nb, tlen), h->pt))) return rc;
  // standalone products: enough workgroups to fill the chip
  int nbs = 64;
  const double w = (double)std::max<int64_t>(h->nnzQ, h->nnzA) + (double)std::max(h->n, h->m);
  while (nbs < 8192 && w / nbs > 2048.0) nbs <<= 1;
  h->nb_spmv = nbs;
  if ((rc = upload_part(h, build_part(h->n, nbs, qlen), h->sq))) return rc;
  if ((rc = upload_part(h, build_part(h->m, nbs, alen), h->sa))) return rc;
  if ((rc = upload_part(h, build_part(h->n, nbs, tlen), h->st_))) return rc;
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
  p.x32 = h->x32; p.r32 = h->r32; p.p32_0 = h->p32_0; p.p32_1 = h->p32_1;
  p.part = h->part;
  p.bar = h->bar;
  p.st = h->st;
  p.pn1 = h->pn1.view();
  p.pcg = h->pcg.view();
  p.pm = h->pm.view();
  const pdhcg_settings& s = h->s;
  p.tol = s.tol_rel_kkt;
  p.eps_factor = s.cg_eps_factor;
  p.beta_suf = s.beta_sufficient;
  p.beta_nec = s.beta_necessary;
  p.beta_art = s.beta_artificial;
  p.theta = s.primal_weight_theta;
  p.eta = s.step_eta_factor / (h->norm_A > 0.0 ? h->norm_A : 1.0);
  p.max_iters = s.max_iters;
  p.iters_this_launch = 5000;
  p.time_limit_ticks = s.time_limit_s > 0.0 ? (uint64_t)(s.time_limit_s * 1e8) : 0;  // 100 MHz clock
  p.max_cg = s.max_cg_iters;
  p.cg_rule = s.cg_rule;
  p.restart_to = s.restart_to;
  p.eval_period = s.eval_period;
  p.mixed_allowed = s.precision == 1;
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
  HIPX(hipMemsetAsync(h->bar, 0, sizeof(uint64_t) * 512, h->stream));
  HIPX(launch_power(pp, h->nb, h->stream));
  double v = 0.0;
  HIPX(hipMemcpyAsync(&v, h->scratch, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
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
  s->verbose = 0;
}

int pdhcg_create(pdhcg_handle** out, const pdhcg_csr* Qc, const pdhcg_csr* Ac, const double* b, const double* c,
                 int32_t vec_on_device, const pdhcg_settings* s, void* hip_stream) {
  const double t0 = now_s();
  if (!out) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle pointer");
  *out = nullptr;
  int rc;
  if ((rc = check_settings(s))) return rc;
  HostCsr Q, A;
  if ((rc = fetch_csr(Qc, Q, "Q"))) return rc;
  if ((rc = fetch_csr(Ac, A, "A"))) return rc;
  if (Q.nrows != Q.ncols) return fail(PDHCG_ERR_INVALID_ARGUMENT, "Q must be square");
  if (A.ncols != Q.nrows) return fail(PDHCG_ERR_INVALID_ARGUMENT, "A must have as many columns as Q");
  if (Q.nrows == 0) return fail(PDHCG_ERR_INVALID_ARGUMENT, "n must be >= 1");
  if (!exactly_symmetric(Q)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "Q is not exactly symmetric");
  if (!c || (A.nrows > 0 && !b)) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null b or c");
  HostCsr T = transpose(A);

  pdhcg_handle* h = new pdhcg_handle();
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

  if ((rc = upload_csr(h, Q, &h->q_rowptr, &h->q_col, &h->q_val))) return bail(rc);
  if ((rc = upload_csr(h, A, &h->a_rowptr, &h->a_col, &h->a_val))) return bail(rc);
  if ((rc = upload_csr(h, T, &h->t_rowptr, &h->t_col, &h->t_val))) return bail(rc);
  const int64_t n = h->n, m = h->m;
  double** nvecs[] = {&h->c, &h->x, &h->xa, &h->x_anc, &h->r, &h->p0, &h->p1, &h->q, &h->tmp_x0};
  for (double** v : nvecs)
    if ((rc = h->alloc(v, n))) return bail(rc);
  double** mvecs[] = {&h->b, &h->y, &h->ya, &h->ax, &h->ax_avg, &h->y_anc, &h->tmp_y0};
  for (double** v : mvecs)
    if ((rc = h->alloc(v, m))) return bail(rc);
  if ((rc = h->alloc(&h->scratch, 16))) return bail(rc);
  if ((rc = h->alloc(&h->part, (int64_t)NSLOT * 4096))) return bail(rc);
  if ((rc = h->alloc(&h->bar, 512))) return bail(rc);
  if ((rc = h->alloc(&h->st, 1))) return bail(rc);
  if ((rc = upload(h, h->b, hb.data(), m))) return bail(rc);
  if ((rc = upload(h, h->c, hc.data(), n))) return bail(rc);
  if ((rc = plan(h, Q, A, T))) return bail(rc);
  if (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess)
    return bail(fail(PDHCG_ERR_HIP, "hipEventCreate failed"));
  if (s->precision == 1 && (rc = ensure_mixed(h))) return bail(rc);
  if ((rc = estimate_norm(h))) return bail(rc);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(PDHCG_ERR_HIP, "stream sync failed"));
  h->setup_s = now_s() - t0;
  if (s->verbose)
    fprintf(stderr, "[pdhcg] n=%lld m=%lld nnzQ=%lld nnzA=%lld nb=%d groups n1=%d q=%d m=%d ||A||=%.6g setup=%.3fs\n",
            (long long)n, (long long)m, (long long)h->nnzQ, (long long)h->nnzA, h->nb, h->pn1.group, h->pcg.group,
            h->pm.group, h->norm_A, h->setup_s);
  *out = h;
  return 0;
}

int pdhcg_set_settings(pdhcg_handle* h, const pdhcg_settings* s) {
  if (!h) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle");
  int rc;
  if ((rc = check_settings(s))) return rc;
  const bool replan = s->num_blocks != h->s.num_blocks;
  const int32_t old_power = h->s.power_iters;
  h->s = *s;
  if (replan) return fail(PDHCG_ERR_INVALID_ARGUMENT, "num_blocks cannot change after pdhcg_create");
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
    HIPX(hipStreamSynchronize(h->stream));
  }
  h->nb_inf = max_abs_nan(hb.data(), h->m);
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
    dx0 = h->tmp_x0;
  }
  if (y0 && h->m > 0) {
    HIPX(hipMemcpyAsync(h->tmp_y0, y0, sizeof(double) * h->m, in_kind, h->stream));
    dy0 = h->tmp_y0;
  }
  SolveParams p = make_params(h);
  SolverState st{};
  st.K_anchor = std::numeric_limits<double>::quiet_NaN();
  st.K_prev = std::numeric_limits<double>::infinity();
  st.omega = h->s.primal_weight_init;
  st.tau = p.eta / st.omega;
  st.sigma = p.eta * st.omega;
  st.mixed = h->s.precision == 1 ? 1 : 0;
  HIPX(hipMemcpyAsync(h->st, &st, sizeof(st), hipMemcpyHostToDevice, h->stream));
  HIPX(launch_init_point(p, dx0, dy0, h->nb, h->stream));
  double kernel_ms = 0.0;
  for (;;) {
    HIPX(hipMemsetAsync(h->bar, 0, sizeof(uint64_t) * 512, h->stream));
    HIPX(hipEventRecord(h->ev0, h->stream));
    HIPX(launch_solve(p, h->nb, h->nb_inf, h->nc_inf, h->stream));
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
  HIPX(hipMemcpyAsync(x_out, h->x, sizeof(double) * h->n, out_kind, h->stream));
  if (h->m > 0) HIPX(hipMemcpyAsync(y_out, h->y, sizeof(double) * h->m, out_kind, h->stream));
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
  }
  return 0;
}

int pdhcg_spmv(pdhcg_handle* h, int32_t which, int32_t precision, const double* x, double* y, int32_t repeats) {
  if (!h || !x || !y) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null argument");
  if (which < 0 || which > 2) return fail(PDHCG_ERR_INVALID_ARGUMENT, "which must be 0 (Q), 1 (A) or 2 (A')");
  if (precision != 0 && precision != 1) return fail(PDHCG_ERR_INVALID_ARGUMENT, "precision must be 0 or 1");
  int rc;
  if (precision == 1 && (rc = ensure_mixed(h))) return rc;
  const DevMat M = h->mat(which);
  if (M.nrows == 0) return 0;
  const DevPart& pt = which == 0 ? h->sq : (which == 1 ? h->sa : h->st_);
  float* x32 = nullptr;
  if (precision == 1) {
    x32 = h->xs32;  // scratch FP32 copy of x
    HIPX(launch_to_f32(x, x32, M.ncols, h->stream));
  }
  for (int r = 0; r < std::max(repeats, 1); ++r)
    HIPX(launch_spmv(M, pt.view(), h->nb_spmv, precision, x, x32, y, h->stream));
  HIPX(hipStreamSynchronize(h->stream));
  return 0;
}

int pdhcg_plan_info(const pdhcg_handle* h, int32_t* num_blocks, int32_t* group_n, int32_t* group_q, int32_t* group_m,
                    int64_t* long_rows) {
  if (!h) return fail(PDHCG_ERR_INVALID_ARGUMENT, "null handle");
  if (num_blocks) *num_blocks = h->nb;
  if (group_n) *group_n = h->pn1.group;
  if (group_q) *group_q = h->pcg.group;
  if (group_m) *group_m = h->pm.group;
  if (long_rows) *long_rows = h->pn1.nlong + h->pcg.nlong + h->pm.nlong;
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

extern "C" int pdhcg_solve_batch(int32_t count, const pdhcg_csr* Qs, const pdhcg_csr* As, const double* const* bs,
                                 const double* const* cs, const double* const* x0s, const double* const* y0s,
                                 double* const* x_outs, double* const* y_outs, pdhcg_result* rs,
                                 const pdhcg_settings* s, void* hip_stream) {
  (void)count; (void)Qs; (void)As; (void)bs; (void)cs; (void)x0s; (void)y0s; (void)x_outs; (void)y_outs;
  (void)rs; (void)s; (void)hip_stream;
  return fail(PDHCG_ERR_INVALID_ARGUMENT, "batched solve kernel not built yet");
}
