/*
 * pdhcg.h -- C ABI of the MI355X (gfx950) restarted PDHCG library.
 *
 * Solves the convex QP  min 1/2 x'Qx + c'x  s.t.  Ax <= b  (problem (1) of
 * Huang et al., "Restarted Primal-Dual Hybrid Conjugate Gradient Method for
 * Large-Scale Quadratic Programming") with Alg. 1 (restarted PDHCG): each
 * iteration solves the proximal primal subproblem inexactly by conjugate
 * gradient, then takes the projected dual step at the extrapolated point,
 * averages the iterates, and restarts adaptively on the relative KKT error
 * (Sec. 4).  Every step of the iteration runs in the library's own HIP
 * kernels on the GPU; the library allocates its device workspace itself.
 *
 * Conventions for every function:
 *  - Return 0 on success or a negative error code (PDHCG_ERR_*).  No C++
 *    exception crosses this boundary.  pdhcg_last_error() gives a message
 *    for the last failure on the calling thread.
 *  - Solve outcomes (converged, iteration or time limit, non-finite values)
 *    are not errors: they are reported in pdhcg_result.status.
 *  - The caller owns every buffer it passes.  pdhcg_create copies the problem
 *    data, so inputs may be freed or reused after it returns.
 *  - Pointers flagged "on_device" point to device memory of the current HIP
 *    device (for example the data_ptr() of a torch tensor); otherwise they are
 *    host pointers.  All device work is issued on the stream given to
 *    pdhcg_create; functions return after that stream has finished the work.
 *  - A handle is not thread-safe.  Separate handles are independent.
 */
#ifndef PDHCG_H
#define PDHCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PDHCG_OK = 0,
    PDHCG_ERR_INVALID_ARGUMENT = -1, /* bad shape, unsorted/duplicate/out-of-range columns,
                                        rowptr not monotone, Q not exactly symmetric, sizes
                                        beyond int32 indexing */
    PDHCG_ERR_OUT_OF_MEMORY = -2,
    PDHCG_ERR_HIP = -3               /* a HIP runtime call or a kernel failed */
};

enum {
    PDHCG_STATUS_OPTIMAL = 0,        /* relKKT <= tol_rel_kkt (Sec. 4 progress metric) */
    PDHCG_STATUS_ITERATION_LIMIT = 1,
    PDHCG_STATUS_TIME_LIMIT = 2,
    PDHCG_STATUS_NUMERICAL_ERROR = 3 /* NaN/Inf appeared; the epoch's anchor point is returned */
};

/* Sparse matrix in CSR form: row i holds entries rowptr[i] .. rowptr[i+1]-1,
 * column indices strictly increasing within a row.  rowptr has nrows+1 entries
 * with rowptr[0] = 0 and rowptr[nrows] = nnz.  Values are FP64. */
typedef struct {
    int64_t nrows, ncols, nnz;
    const int64_t* rowptr;
    const int32_t* col;
    const double* val;
    int32_t on_device;               /* 1: the three arrays are device pointers */
} pdhcg_csr;

/* Solver settings.  pdhcg_default_settings fills the defaults noted here. */
typedef struct {
    double tol_rel_kkt;              /* 1e-4; stop when relKKT <= tol (Sec. 4, progress metric) */
    int64_t max_iters;               /* 100000; cap on PDHCG iterations (inner steps, all epochs) */
    int32_t max_cg_iters;            /* 100; N, the CG step cap per iteration (Sec. 2) */
    int32_t cg_rule;                 /* 0: adaptive epsilon_k tolerance (Sec. 4), 1: always N steps
                                        (PDHCG-fixed, Thm 1); N = 1 gives a linearised primal step */
    double cg_eps_factor;            /* 0.05: epsilon_k = epsilon_{k-1} + 0.05 relKKT (Sec. 4) */
    double beta_sufficient;          /* 0.2  (Sec. 4, adaptive restart) */
    double beta_necessary;           /* 0.8 */
    double beta_artificial;          /* 0.2 */
    int32_t restart_to;              /* 0: better of current and average, 1: average (Alg. 1) */
    int32_t eval_period;             /* 64: iterations between restart evaluations */
    double primal_weight_theta;      /* 0.2 (Sec. 4, primal weight adjustment); 0 freezes omega */
    double primal_weight_init;       /* 1.0 */
    double step_eta_factor;          /* 0.5: eta = 0.5/||A||_2, tau = eta/omega, sigma = eta*omega
                                        (sigma = tau = 1/(2||A||) at omega = 1, Thm 2) */
    int32_t power_iters;             /* 100: power-iteration steps for ||A||_2 */
    int32_t precision;               /* 0: FP64 throughout.  1: FP32 matrix values and FP32 copies
                                        of the vectors in the CG and dual-step products, FP64
                                        accumulation, FP64 scalars, FP64 relKKT; termination is
                                        certified against the FP64 data */
    double time_limit_s;             /* 0 = none */
    int32_t num_blocks;              /* 0 = planner's choice; else workgroups of the solve kernel */
    int32_t warm_fallback;           /* 1: if relKKT at a given (x0, y0) exceeds relKKT at (0, 0),
                                        start from (0, 0) instead (a cold start) */
    int32_t verbose;                 /* 0 = silent */
    int32_t cg_form;                 /* form of the CG steps in the single-QP solve (same iterates
                                        in exact arithmetic): 0 = planner's choice (1 while the
                                        interleaved FP32 (r, u, s) vector, 16 n bytes, fits the L2
                                        of one XCD, else 2), 1 = one reduction and one grid barrier
                                        per step with (r, u, s) gathered (Chronopoulos-Gear),
                                        2 = textbook CG, two barriers per step with only the
                                        direction gathered */
    int32_t ruiz_iters;              /* 0 (off); diagonal preconditioning (Sec. 4, preprocessing):
                                        Ruiz equilibration steps on K = [[Q, A'], [A, 0]], the paper
                                        runs 10.  The solver then iterates on D2 Q D2, D1 A D2, D1 b,
                                        D2 c, while relKKT, the residuals, the termination, the CG
                                        tolerance schedule and the restart tests are those of the
                                        caller's problem at x = D2 x~, y = D1 y~ (the progress metric
                                        is defined for problem (1) as posed); x and y of the caller's
                                        problem are returned.  Fixed
                                        at pdhcg_create for a handle; the batched entry points scale
                                        every instance on its own (its Q and A are then stored
                                        unshared; a factored Q keeps its factor form) */
    int32_t pock_chambolle;          /* 0 (off); 1: one Pock-Chambolle step (alpha = 1) after the
                                        Ruiz steps; same rules as ruiz_iters */
    int32_t step_rule;               /* 0: constant eta per epoch (Thm 2; changed only through the
                                        primal weight).  1: adaptive step size (Sec. 4): each
                                        iteration's primal and dual steps are a trial at the current
                                        eta, accepted when eta <= eta_bar = ||dz||_w^2 /
                                        (2 |dy'A dx| + dx'Q dx) (||.||_w the primal-weight norm);
                                        eta becomes min((1 - (t+1)^-0.3) eta_bar, (1 + (t+1)^-0.6) eta)
                                        after every trial, and a rejected trial is repeated from
                                        z^k.  eta starts at step_eta_factor / ||A||_2 and persists
                                        across restarts.  The single-QP solve then keeps its CG
                                        state in device memory (no chained steps) */
    int32_t threads;                 /* threads per workgroup of the single-QP solve and power
                                        kernels: 0 = planner's choice (256, two workgroups per CU,
                                        once the gathered vectors outgrow the L2 of one XCD,
                                        12 n bytes, for a sparse Q; else 512, one per CU), 256
                                        or 512.  Every setting computes the same iterates up to
                                        the order of the FP64 reductions (the row partitions
                                        follow the workgroup count) */
} pdhcg_settings;

typedef struct {
    int32_t status;                  /* PDHCG_STATUS_* */
    int32_t returned_average;        /* 1 if the running average was returned */
    double rel_primal, rel_dual, rel_gap, rel_kkt;  /* of the returned point, FP64 data */
    double primal_obj, dual_obj;     /* 1/2 x'Qx + c'x and -1/2 x'Qx - b'y */
    int64_t iters;                   /* PDHCG iterations */
    int64_t cg_iters_total;          /* CG steps over all iterations */
    int64_t restarts;
    double norm_A;                   /* power-iteration estimate of ||A||_2 */
    double setup_s;                  /* wall time of pdhcg_create */
    double solve_s;                  /* wall time of the solve */
    double kernel_s;                 /* device time of the solve kernel launches (HIP events on the
                                        handle's stream) */
    int64_t kkt_evals;               /* restart evaluations (relKKT of the average) performed */
    int32_t cold_fallback;           /* 1 if the given start point was replaced by (0, 0) */
    int64_t rejected_steps;          /* trials rejected by the adaptive step size (step_rule 1) */
    double step_eta;                 /* eta at the end of the solve */
    int64_t qx_formed;               /* n-side passes at the current point that formed Q x with a
                                        product: one per iteration, except in the batch with a dense
                                        or factored Q and the constant step rule, where Q x is kept
                                        by linearity through the CG updates and formed only at the
                                        start, every eval_period iterations, after a restart to the
                                        average and before a termination or a limit is reported */
} pdhcg_result;

typedef struct pdhcg_handle pdhcg_handle;

void pdhcg_default_settings(pdhcg_settings* s);

/* Copy the problem to the device, build A' (CSR), plan the kernels' row
 * partitions, and estimate ||A||_2.  Q (n x n) must hold both triangles and
 * be exactly symmetric; A is m x n (m may be 0).  b (m) and c (n) are FP64,
 * on the device when vec_on_device = 1.  hip_stream may be NULL (the default
 * stream).  On success *h owns all device memory of the problem. */
int pdhcg_create(pdhcg_handle** h, const pdhcg_csr* Q, const pdhcg_csr* A, const double* b,
                 const double* c, int32_t vec_on_device, const pdhcg_settings* s, void* hip_stream);

/* A QP whose Q is given in low-rank form, Q = P P' + diag(d) (Sec. 2,
 * low-rank acceleration of Q): P is a sparse n x k CSR matrix (k >= 1, FP64
 * values), d (n entries, finite and >= 0) may be NULL for d = 0.  Every product with Q is formed as t = P' v, then
 * P t + d v (P' is built and stored beside P at create time), so a CG step
 * reads nnz(P) twice instead of nnz(P P'); that product takes one more grid
 * barrier.  A, b, c, settings, stream and errors as pdhcg_create; d is a
 * device pointer when vec_on_device = 1.  The handle then solves with the
 * textbook CG form, without diagonal preconditioning and with the constant
 * step rule (ruiz_iters, pock_chambolle and step_rule must be 0:
 * INVALID_ARGUMENT otherwise), and pdhcg_spmv takes which = 1 or 2 only. */
int pdhcg_create_lowrank(pdhcg_handle** h, const pdhcg_csr* P, const double* d, const pdhcg_csr* A,
                         const double* b, const double* c, int32_t vec_on_device, const pdhcg_settings* s,
                         void* hip_stream);

/* Replace the settings of a handle (e.g. a different tolerance or CG cap). */
int pdhcg_set_settings(pdhcg_handle* h, const pdhcg_settings* s);

/* Replace b (length m) of an existing problem, keeping Q, A, c and the plan
 * (used for a family of QPs that differ only in b). */
int pdhcg_set_b(pdhcg_handle* h, const double* b, int32_t vec_on_device);

/* Run restarted PDHCG from (x0, y0) (NULL = zero; y0 is projected onto
 * y >= 0) and write the returned point to x_out (n) and y_out (m).  Vectors
 * are device pointers when vec_on_device = 1.  r may be NULL. */
int pdhcg_solve(pdhcg_handle* h, const double* x0, const double* y0, double* x_out, double* y_out,
                int32_t vec_on_device, pdhcg_result* r);

/* Solve `count` independent QPs in one call (pdhcg_batch_create, one
 * pdhcg_batch_solve, pdhcg_batch_destroy).  The CSR matrices may be host or
 * device arrays (their on_device flags); bs, cs, x0s, y0s, x_outs, y_outs are
 * host arrays.  Every instance is solved by one workgroup of a persistent
 * kernel and gets its own status in rs[i].  x0s/y0s may be NULL (cold start)
 * or hold NULL entries. */
int pdhcg_solve_batch(int32_t count, const pdhcg_csr* Qs, const pdhcg_csr* As,
                      const double* const* bs, const double* const* cs,
                      const double* const* x0s, const double* const* y0s,
                      double* const* x_outs, double* const* y_outs, pdhcg_result* rs,
                      const pdhcg_settings* s, void* hip_stream);

/* Bytes of the static device array behind pdhcg_solve_batch_noalloc (one copy
 * per GPU the library runs on, held until the process ends). */
#define PDHCG_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (serving loops and
 * harnesses that forbid hipMalloc): pdhcg_solve_batch with the same
 * arguments, results and errors, except that every device buffer of the
 * batch (packed matrices and vectors, row partitions, parameter blocks,
 * per-instance state, preconditioning factors) is carved from a static device
 * array of PDHCG_NOALLOC_SCRATCH_BYTES instead of being allocated; no
 * hipMalloc, hipFree or allocating library routine is called (host memory is
 * still used for packing).  A batch that does not fit returns
 * PDHCG_ERR_INVALID_ARGUMENT with the bytes it needs in pdhcg_last_error().
 * Every call on a GPU shares that GPU's array, so calls that overlap on one
 * GPU (other threads, other streams) race and must be serialised by the
 * caller; a call returns after its stream has finished using the array.
 * kernel_s in rs is the solve's host wall time, as solve_s (no events are
 * created).  The call synchronizes its stream, so it cannot be captured into
 * a HIP graph. */
int pdhcg_solve_batch_noalloc(int32_t count, const pdhcg_csr* Qs, const pdhcg_csr* As,
                              const double* const* bs, const double* const* cs,
                              const double* const* x0s, const double* const* y0s,
                              double* const* x_outs, double* const* y_outs, pdhcg_result* rs,
                              const pdhcg_settings* s, void* hip_stream);

/* A dense Q given by its factor: Q = F F' + diag(d), F n x k (row-major,
 * k <= n), d (n).  The low-rank form of Q (Sec. 2, low-rank acceleration; the
 * portfolio model of Sec. 5.1): the batched products then read 2 n k values
 * per product instead of n^2. */
typedef struct {
    int64_t n, k;
    const double* F;
    const double* d;
    int32_t on_device;               /* 1: F and d are device pointers */
} pdhcg_lowrank;

/* pdhcg_solve_batch with every Q given by its factor (Qs[i]); A, b, c, start
 * points, outputs, results and errors as there.  The products apply
 * t = F' v, then F t + d v (two streamed passes over F and its transpose,
 * which the library stores beside it). */
int pdhcg_solve_batch_lowrank(int32_t count, const pdhcg_lowrank* Qs, const pdhcg_csr* As,
                              const double* const* bs, const double* const* cs,
                              const double* const* x0s, const double* const* y0s,
                              double* const* x_outs, double* const* y_outs, pdhcg_result* rs,
                              const pdhcg_settings* s, void* hip_stream);

/* Solve `count` QPs that share Q, A and c and differ only in b (one family
 * with many right-hand sides, e.g. the training data of a learned warm
 * start): B holds b_i at B + i*m (m x count, column i = instance i), X0/Y0
 * (may be NULL) hold the start points the same way (n x count, m x count), and
 * X/Y receive the returned points (n x count, m x count).  All host arrays.
 * The same batched kernel as pdhcg_solve_batch, with Q and A uploaded once;
 * rs[i] is instance i's result.  Errors as pdhcg_solve_batch. */
int pdhcg_solve_multi_rhs(int32_t count, const pdhcg_csr* Q, const pdhcg_csr* A, const double* B,
                          const double* c, const double* X0, const double* Y0, double* X, double* Y,
                          pdhcg_result* rs, const pdhcg_settings* s, void* hip_stream);

/* ----------------------------------------------------------------- batches
 * A batch of independent QPs packed into device memory once and solved any
 * number of times (Alg. 1 on every instance, one workgroup per instance).
 * Vectors of the instances are packed end to end: x of instance i occupies
 * entries n_off[i] .. n_off[i+1]-1 of a packed n-vector, y of instance i
 * entries m_off[i] .. m_off[i+1]-1 of a packed m-vector (pdhcg_batch_layout). */
typedef struct pdhcg_batch pdhcg_batch;

/* Validate, pack and upload `count` QPs.  Exactly one of Qs (CSR; a dense
 * n x n pattern is detected and stored as a dense block) and Ls (factors of
 * Q = F F' + diag(d)) is non-NULL.  CSR and factor arrays are device or host
 * arrays by their own on_device flags; bs[i] (m_i) and cs[i] (n_i) are device
 * pointers when vec_on_device = 1.  Matrices given by the same pointers are
 * stored once (not with preconditioning, which scales every instance on its
 * own in one launch).  The caller's arrays may be freed afterwards.  Errors:
 * INVALID_ARGUMENT (null pointers, bad shapes, CSR structure, Q not exactly
 * symmetric), OUT_OF_MEMORY, HIP; on error *h is NULL. */
int pdhcg_batch_create(pdhcg_batch** h, int32_t count, const pdhcg_csr* Qs, const pdhcg_lowrank* Ls,
                       const pdhcg_csr* As, const double* const* bs, const double* const* cs,
                       int32_t vec_on_device, const pdhcg_settings* s, void* hip_stream);

/* n_off and m_off (count + 1 entries each) receive the packed offsets. */
int pdhcg_batch_layout(const pdhcg_batch* h, int64_t* n_off, int64_t* m_off);

/* Solve every instance from the packed start points x0 / y0 (NULL: cold
 * start (0, 0); y0 is projected onto y >= 0) and write the returned points to
 * the packed x_out / y_out.  All four are device pointers when
 * vec_on_device = 1, else host pointers.  rs (count entries, may be NULL)
 * receives each instance's result; kernel_s is the device time of the one
 * batched launch.  Solve outcomes are per instance (rs[i].status). */
int pdhcg_batch_solve(pdhcg_batch* h, const double* x0, const double* y0, double* x_out, double* y_out,
                      int32_t vec_on_device, pdhcg_result* rs);

/* Threads per workgroup of the batch's kernel: 256 (the default: two
 * instances per CU, LDS tiles of 2 048 entries and 512 rows) or 512 (one
 * instance per CU, tiles of 4 096 entries and 1 024 rows).  A batch made by
 * pdhcg_batch_create holds the row partitions for both; the result of a solve
 * differs between the two only in the rounding of its reductions.
 * INVALID_ARGUMENT for another value. */
int pdhcg_batch_set_threads(pdhcg_batch* h, int32_t threads);

/* Autotuner of the batched kernel: solve every instance of the batch from a
 * cold start `reps` times with each workgroup size (256 and 512 threads, with
 * their tile sizes) and keep the faster for later solves.  *threads receives
 * the choice; kernel_s (2 entries, may be NULL) the fastest launch time of
 * each candidate in seconds, 256 first.  The returned points and results of
 * these solves are discarded.  INVALID_ARGUMENT for reps < 1 or a null
 * handle; HIP on a failed launch. */
int pdhcg_batch_autotune(pdhcg_batch* h, int32_t reps, int32_t* threads, double* kernel_s);

/* The packed D1 (rows) and D2 (variables) of the batch's preconditioning
 * (ones when it is off); device pointers when vec_on_device = 1. */
int pdhcg_batch_get_scaling(const pdhcg_batch* h, double* d1_out, double* d2_out, int32_t vec_on_device);

void pdhcg_batch_destroy(pdhcg_batch* h);

/* The diagonals of the preconditioning of a handle (Sec. 4, preprocessing):
 * d1_out[m] = D1 (constraint rows), d2_out[n] = D2 (variables); all ones when
 * ruiz_iters = 0 and pock_chambolle = 0 at pdhcg_create.  Outputs are device
 * pointers when vec_on_device = 1, else host pointers; d1_out may be NULL when
 * m = 0.  Returns INVALID_ARGUMENT for a null handle or output. */
int pdhcg_get_scaling(const pdhcg_handle* h, double* d1_out, double* d2_out, int32_t vec_on_device);

/* y = M x with the library's SpMV kernel on the handle's device copy of
 * M = Q (which = 0), A (1) or A' (2), in FP64 (precision 0) or with FP32
 * values and an FP32 copy of x (precision 1, FP64 accumulation).  x and y are
 * FP64 device pointers.  repeats > 1 launches the same product back to back
 * (for timing).  With preconditioning on, M is the scaled matrix.  Test and
 * measurement entry point. */
int pdhcg_spmv(pdhcg_handle* h, int32_t which, int32_t precision, const double* x, double* y,
               int32_t repeats);

/* Autotuner of the single-QP kernel: for each workgroup size (512 and 256
 * threads), candidate grid size (64, 128, 256, 512 workgroups, within what
 * stays co-resident at that size) and lane-group scaling (the planner's lane
 * group per row halved, as planned, doubled) run `iters` iterations from
 * (0, 0) and time the solve kernel (HIP events); keep the fastest per
 * iteration and re-plan the row partitions for it.  The settings' num_blocks
 * and threads become the chosen grid and workgroup sizes (pdhcg_plan_info
 * reports both).  num_blocks and group_scale (log2 of the scaling) may be
 * NULL. */
int pdhcg_autotune(pdhcg_handle* h, int32_t iters, int32_t* num_blocks, int32_t* group_scale);

/* Grid size, row-split parameters and threads per workgroup of the
 * cooperative kernels that the planner chose (for reporting); any output may
 * be NULL. */
int pdhcg_plan_info(const pdhcg_handle* h, int32_t* num_blocks, int32_t* group_n, int32_t* group_q,
                    int32_t* group_m, int64_t* long_rows, int32_t* threads);

void pdhcg_destroy(pdhcg_handle* h);

const char* pdhcg_error_string(int code);
const char* pdhcg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PDHCG_H */
