/*
 * FP64 CPU reference of restarted PDHCG for  min 1/2 x'Qx + c'x  s.t.  Ax <= b.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the GPU library, and the GPU library never calls it.
 *
 * It is written to be read next to the paper (Huang et al., "Restarted
 * Primal-Dual Hybrid Conjugate Gradient Method for Large-Scale Quadratic
 * Programming"): plain CSR loops, double precision everywhere, no blocking or
 * fusion.  Each function names the passage it follows.  Readings of passages
 * that are silent, garbled or ambiguous are marked READING and are the same
 * readings the GPU library implements (they are listed in the design notes).
 *
 * Parity status: every function is pinned by CPU tests against closed forms,
 * brute force or library routines, except the whole solve on generic
 * generated instances, whose only pin is its own KKT residual (no closed form
 * exists there).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int64_t nrows, ncols;
    const int64_t* rowptr;
    const int32_t* col;
    const double* val;
} or_csr;

/* Mirrors the fields of the library's settings one to one (own definition). */
typedef struct {
    double tol;               /* relKKT termination tolerance (Sec. 4, progress metric) */
    int64_t max_iters;        /* cap on PDHCG iterations (inner steps, all epochs) */
    int32_t max_cg;           /* N: CG step cap per iteration (PDHCG-fixed, Sec. 2) */
    int32_t cg_rule;          /* 0: adaptive tolerance, 1: always N steps */
    double cg_eps_factor;     /* 0.05 in the epsilon_k schedule (Sec. 4, BB/CG paragraph) */
    double beta_suf, beta_nec, beta_art;  /* 0.2, 0.8, 0.2 (Sec. 4, adaptive restart) */
    int32_t restart_to;       /* 0: better of current/average, 1: average (Alg. 1) */
    int32_t eval_period;      /* iterations between restart evaluations */
    double pw_theta;          /* 0.2 (Sec. 4, primal weight adjustment); 0 = frozen */
    double pw_init;           /* initial primal weight */
    double eta_factor;        /* eta = eta_factor / ||A||_2 (sigma = tau = 1/(2||A||), Thm 2) */
    int32_t power_iters;      /* power-iteration steps for ||A||_2 */
    int32_t step_rule;        /* 0: constant eta per epoch (Thm 2), 1: adaptive step (Sec. 4) */
} or_settings;

/* ---------------------------------------------------------------- basics */

/* y = M x, one row at a time. */
void or_matvec(const or_csr* M, const double* x, double* y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < M->nrows; ++i) {
        double s = 0.0;
        for (int64_t k = M->rowptr[i]; k < M->rowptr[i + 1]; ++k) s += M->val[k] * x[M->col[k]];
        y[i] = s;
    }
}

/* x = M' y, by scattering each row of M. */
void or_matvec_t(const or_csr* M, const double* y, double* x) {
    for (int64_t j = 0; j < M->ncols; ++j) x[j] = 0.0;
    for (int64_t i = 0; i < M->nrows; ++i)
        for (int64_t k = M->rowptr[i]; k < M->rowptr[i + 1]; ++k) x[M->col[k]] += M->val[k] * y[i];
}

static double dot(int64_t n, const double* a, const double* b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* max that propagates NaN (fmax would drop it and hide a diverged iterate) */
static double maxp(double a, double b) {
    if (isnan(a) || isnan(b)) return NAN;
    return a > b ? a : b;
}

static double norm_inf(int64_t n, const double* a) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s = maxp(s, fabs(a[i]));
    return s;
}

static double dist2(int64_t n, const double* a, const double* b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += (a[i] - b[i]) * (a[i] - b[i]);
    return sqrt(s);
}

static double* alloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

/* ---------------------------------------------------------------- relKKT */

/*
 * Relative KKT error (Sec. 4, "Progress metric"):
 *   r_primal = ||[Ax - b]^+||_inf / (1 + max(||Ax||_inf, ||b||_inf))
 *   r_dual   = ||Qx + A'y + c||_inf / (1 + max(||Qx||_inf, ||A'y||_inf, ||c||_inf))
 *   r_gap    = |x'Qx + c'x + b'y| / (1 + max(|1/2 x'Qx + c'x|, |1/2 x'Qx + b'y|))
 *   relKKT   = max of the three.
 * out[0..7] = r_primal, r_dual, r_gap, relKKT, primal objective
 *             1/2 x'Qx + c'x, dual objective -1/2 x'Qx - b'y, x'Qx, b'y.
 */
void or_kkt(const or_csr* Q, const or_csr* A, const double* b, const double* c,
            const double* x, const double* y, double* out) {
    int64_t n = Q->nrows, m = A->nrows;
    double* Qx = alloc(n);
    double* Aty = alloc(n);
    double* Ax = alloc(m);
    or_matvec(Q, x, Qx);
    or_matvec_t(A, y, Aty);
    or_matvec(A, x, Ax);
    double viol = 0.0;
    for (int64_t i = 0; i < m; ++i) viol = maxp(viol, maxp(Ax[i] - b[i], 0.0));
    double r_p = viol / (1.0 + maxp(norm_inf(m, Ax), norm_inf(m, b)));
    double dres = 0.0;
    for (int64_t j = 0; j < n; ++j) dres = maxp(dres, fabs(Qx[j] + Aty[j] + c[j]));
    double r_d = dres / (1.0 + maxp(norm_inf(n, Qx), maxp(norm_inf(n, Aty), norm_inf(n, c))));
    double xQx = dot(n, x, Qx), cx = dot(n, c, x), by = dot(m, b, y);
    double r_g = fabs(xQx + cx + by) / (1.0 + maxp(fabs(0.5 * xQx + cx), fabs(0.5 * xQx + by)));
    out[0] = r_p;
    out[1] = r_d;
    out[2] = r_g;
    out[3] = maxp(r_p, maxp(r_d, r_g));
    out[4] = 0.5 * xQx + cx;
    out[5] = -0.5 * xQx - by;
    out[6] = xQx;
    out[7] = by;
    free(Qx);
    free(Aty);
    free(Ax);
}

/*
 * The caller's problem when the solve runs on a diagonally preconditioned copy
 * (Sec. 4, "Preprocessing"): the iterates live in the scaled problem
 * Q~ = D2 Q D2, A~ = D1 A D2, b~ = D1 b, c~ = D2 c, and a scaled point
 * (x~, y~) stands for x = D2 x~, y = D1 y~ of problem (1).
 * READING: the progress metric is defined for problem (1) as posed, so every
 * relKKT the method uses (termination, the epsilon_k schedule of the CG, the
 * restart tests) is that of the caller's problem at the mapped point.
 */
typedef struct {
    const or_csr* Q;
    const or_csr* A;
    const double* b;
    const double* c;
    const double* d1;   /* m entries */
    const double* d2;   /* n entries */
} or_original;

/* relKKT pieces of the point (x, y) of the problem the solve iterates on:
 * or_kkt on that problem, or, with `o`, on the caller's problem at
 * (D2 x, D1 y); xm (n) and ym (m) are work space. */
static void kkt_at(const or_csr* Q, const or_csr* A, const double* b, const double* c, const or_original* o,
                   const double* x, const double* y, double* out, double* xm, double* ym) {
    if (!o) {
        or_kkt(Q, A, b, c, x, y, out);
        return;
    }
    for (int64_t j = 0; j < Q->nrows; ++j) xm[j] = o->d2[j] * x[j];
    for (int64_t i = 0; i < A->nrows; ++i) ym[i] = o->d1[i] * y[i];
    or_kkt(o->Q, o->A, o->b, o->c, xm, ym, out);
}

/* ------------------------------------------------------ operator norm of A */

/*
 * ||A||_2, needed by the step sizes sigma = tau = 1/(2||A||) (Thm 2).  The paper
 * does not say how it is obtained.  READING: power iteration on A'A from the
 * fixed start v_j = 0.5 + ((j * 40503) mod 1024) / 1024, normalised; after
 * `iters` steps ||A|| ~ sqrt(||A'A v||) with ||v|| = 1.  Returns 0 for A = 0.
 */
double or_opnorm(const or_csr* A, int32_t iters) {
    int64_t n = A->ncols, m = A->nrows;
    if (m == 0 || n == 0) return 0.0;
    double* v = alloc(n);
    double* w = alloc(n);
    double* Av = alloc(m);
    for (int64_t j = 0; j < n; ++j) v[j] = 0.5 + (double)(((uint64_t)j * 40503u) % 1024u) / 1024.0;
    double nv = sqrt(dot(n, v, v));
    for (int64_t j = 0; j < n; ++j) v[j] /= nv;
    double lam = 0.0;
    for (int32_t it = 0; it < iters; ++it) {
        or_matvec(A, v, Av);
        or_matvec_t(A, Av, w);
        lam = sqrt(dot(n, w, w));
        if (lam == 0.0) break;
        for (int64_t j = 0; j < n; ++j) v[j] = w[j] / lam;
    }
    free(v);
    free(w);
    free(Av);
    return sqrt(lam);
}

/* ------------------------------------------------------------------- CG */

/*
 * Inexact CG for the primal subproblem of Alg. 1:
 *   x+ ~ argmin 1/2 x'Qx + c'x + y'Ax + ||x - xk||^2/(2 tau),
 * i.e. (Q + I/tau) x = xk/tau - c - A'y, started at x = xk.  `g` is
 * Q xk + A'y + c on entry, so the starting residual is r0 = -g.
 * Stopping (Sec. 2, CG stopping criterion; Sec. 4 epsilon_k schedule).
 * READING: the distance to the subproblem optimum is certified by the
 * residual, ||x_l - x*|| <= tau ||r_l|| since the smallest eigenvalue of
 * Q + I/tau is at least 1/tau; CG stops after step l when tau ||r_l|| <= eps,
 * or when l = max_steps (cg_rule 1: always max_steps).  At least one step is
 * taken unless r0 = 0.  x is updated in place; returns the number of steps.
 */
int32_t or_cg(const or_csr* Q, double tau, const double* g, double* x, double eps,
              int32_t max_steps, int32_t cg_rule) {
    int64_t n = Q->nrows;
    double* r = alloc(n);
    double* p = alloc(n);
    double* q = alloc(n);
    for (int64_t j = 0; j < n; ++j) r[j] = -g[j];
    for (int64_t j = 0; j < n; ++j) p[j] = r[j];
    double rho = dot(n, r, r);
    int32_t steps = 0;
    if (rho > 0.0) {
        for (int32_t l = 1; l <= max_steps; ++l) {
            or_matvec(Q, p, q);
            for (int64_t j = 0; j < n; ++j) q[j] += p[j] / tau;
            double alpha = rho / dot(n, p, q);
            for (int64_t j = 0; j < n; ++j) x[j] += alpha * p[j];
            for (int64_t j = 0; j < n; ++j) r[j] -= alpha * q[j];
            double rho_new = dot(n, r, r);
            steps = l;
            if (l == max_steps) break;
            if (cg_rule == 0 && tau * sqrt(rho_new) <= eps) break;
            if (rho_new == 0.0) break;
            double beta = rho_new / rho;
            for (int64_t j = 0; j < n; ++j) p[j] = r[j] + beta * p[j];
            rho = rho_new;
        }
    }
    free(r);
    free(p);
    free(q);
    return steps;
}

/* ------------------------------------------------- restart and weighting */

/*
 * Adaptive restart test (Sec. 4, adaptive restart: the three-condition scheme
 * the paper adopts, with beta_sufficient, beta_necessary, beta_artificial).
 * READING (the conditions themselves are delegated to another paper): with
 * K_c the relKKT of the restart candidate, K_anchor that of the point the
 * current epoch started from, K_prev the candidate's relKKT at the previous
 * evaluation of this epoch (+inf if none), k the iterations in this epoch and
 * k_total all iterations so far, restart if
 *   (i)   K_c <= beta_suf * K_anchor,                    or
 *   (ii)  K_c <= beta_nec * K_anchor and K_c > K_prev,   or
 *   (iii) k >= beta_art * k_total.
 * Returns 1, 2 or 3 for the first condition that holds, 0 for no restart.
 */
int32_t or_restart_decision(double K_c, double K_anchor, double K_prev, int64_t k, int64_t k_total,
                            double beta_suf, double beta_nec, double beta_art) {
    if (K_c <= beta_suf * K_anchor) return 1;
    if (K_c <= beta_nec * K_anchor && K_c > K_prev) return 2;
    if ((double)k >= beta_art * (double)k_total) return 3;
    return 0;
}

/*
 * Primal weight update at a restart (Sec. 4, primal weight adjustment).
 * READING: the printed rule mixes a logarithm with a linear term; the
 * geometric smoothing omega' = exp(theta log(dy/dx) + (1 - theta) log omega)
 * is used, left unchanged unless dx, dy > 1e-10.
 */
double or_primal_weight(double omega, double dx, double dy, double theta) {
    if (dx > 1e-10 && dy > 1e-10) return exp(theta * log(dy / dx) + (1.0 - theta) * log(omega));
    return omega;
}

/* ------------------------------------------------------ adaptive step size */

/*
 * Step-size limit of the adaptive step (Sec. 4, "Adaptive step-size"): for a
 * trial step from z = (x, y) to z' = (x', y'),
 *   eta_bar = ||z' - z||_w^2 / (2 |(x' - x)' A' (y' - y)| + (x' - x)' Q (x' - x)),
 * with ||(dx, dy)||_w^2 = omega ||dx||^2 + ||dy||^2 / omega (the primal-weight
 * norm of the cited PDLP rule, whose limit the paper extends by the Q term).
 * READING: the bilinear term enters with its magnitude, as in the PDLP rule
 * (the paper's sign convention for y makes the printed sign ambiguous); a zero
 * denominator gives +inf.  (The augmented penalty is not used: rho = 0.)
 */
double or_step_limit(const or_csr* Q, const or_csr* A, const double* x, const double* xn, const double* y,
                     const double* yn, double omega) {
    int64_t n = Q->nrows, m = A->nrows;
    double* dx = alloc(n);
    double* dy = alloc(m);
    double* Qdx = alloc(n);
    double* Adx = alloc(m);
    for (int64_t j = 0; j < n; ++j) dx[j] = xn[j] - x[j];
    for (int64_t i = 0; i < m; ++i) dy[i] = yn[i] - y[i];
    or_matvec(Q, dx, Qdx);
    or_matvec(A, dx, Adx);
    double num = omega * dot(n, dx, dx) + dot(m, dy, dy) / omega;
    double den = 2.0 * fabs(dot(m, dy, Adx)) + dot(n, dx, Qdx);
    free(dx); free(dy); free(Qdx); free(Adx);
    return den > 0.0 ? num / den : INFINITY;
}

/*
 * The step size after an attempt at the t-th iteration (t >= 1, counting the
 * iteration being taken), by the update of the cited PDLP rule:
 *   eta' = min((1 - (t + 1)^-0.3) eta_bar, (1 + (t + 1)^-0.6) eta).
 * The attempt is accepted when eta <= eta_bar; either way eta' is the step
 * of the next attempt or iteration.  READING: the exponents and the update are
 * the PDLP rule the paper says it follows; t counts from 1 so that the first
 * factor is positive.
 */
double or_next_step(double eta, double eta_bar, int64_t t) {
    double a = (1.0 - pow((double)t + 1.0, -0.3)) * eta_bar;
    double b = (1.0 + pow((double)t + 1.0, -0.6)) * eta;
    return a < b ? a : b;
}

/* ---------------------------------------------------------------- solve */

enum { OR_OPTIMAL = 0, OR_ITER_LIMIT = 1, OR_NUMERICAL = 3 };

/*
 * Restarted PDHCG (Alg. 1) with the practical rules of Sec. 4.
 *
 * Per iteration k of an epoch (z = (x, y) is z^{n,k}):
 *   K = relKKT(z); stop (OPTIMAL, current point) if K <= tol.
 *   Every eval_period iterations of the epoch: K_avg = relKKT(average);
 *     stop (OPTIMAL, average) if K_avg <= tol; otherwise take the restart
 *     candidate and apply the restart test; on restart update the primal
 *     weight, move to the candidate and start a new epoch.
 *   eps += cg_eps_factor * K                      (epsilon_k schedule, Sec. 4)
 *   x+ = CG on the proximal subproblem from x      (Alg. 1 primal step)
 *   y+ = max(0, y + sigma (A(2x+ - x) - b))       (Alg. 1 dual step; READING:
 *        the sign inside the projection follows the Lagrangian (2), whose
 *        gradient in y is Ax - b, and the appendix's resolvent form)
 *   averages: READING beta_k = k + 1, so the average after k+1 iterations is
 *        the uniform mean of z^{n,1}..z^{n,k+1} (the appendix's average)
 *   k += 1.
 * Step sizes: eta = eta_factor/||A||, tau = eta/omega, sigma = eta*omega
 * (sigma = tau = 1/(2||A||) at omega = 1, Thm 2); ||A|| = 0 is treated as 1.
 * At the iteration cap the point of lower relKKT (current or average) is
 * returned with ITER_LIMIT.  A non-finite relKKT returns the epoch's anchor
 * with NUMERICAL_ERROR.
 *
 * With step_rule = 1 the step size adapts (Sec. 4, "Adaptive step-size"): each
 * iteration's primal and dual steps are a trial at the current eta; the trial
 * is accepted when eta <= or_step_limit of it, and eta becomes or_next_step
 * either way, so a rejected trial is repeated from z^k (the CG from x^k with
 * the new tau) with the smaller step.  tau = eta/omega, sigma = eta*omega as in
 * the constant rule; eta starts at eta_factor/||A|| and persists across
 * restarts.  CG steps of rejected trials count in the CG total.
 *
 * info[0..12]: status, iterations, total CG steps, restarts, returned_average,
 *   r_primal, r_dual, r_gap, relKKT, primal obj, dual obj, ||A|| estimate,
 *   rejected trial steps.
 * With `orig` (may be NULL) the data passed are a preconditioned copy of the
 * caller's problem and every relKKT is taken on the caller's problem at the
 * mapped point (see or_original); the reported r_*, relKKT and objectives are
 * then those of the caller's problem, while x_out, y_out stay scaled.
 * trace_len > 0 records x, y and the running averages after each of the first
 * trace_len iterations (trace_x, trace_xa: trace_len*n; trace_y, trace_ya:
 * trace_len*m), the CG steps of each (trace_cg: trace_len) and, when
 * trace_step is not NULL, the step size of the accepted trial, its limit
 * eta_bar (+inf with the constant rule) and the attempts taken (trace_step:
 * 3*trace_len), for tests of the first steps and of invariants.
 */
int32_t or_solve(const or_csr* Q, const or_csr* A, const double* b, const double* c,
                 const or_settings* s, const double* x0, const double* y0,
                 double* x_out, double* y_out, double* info,
                 int64_t trace_len, double* trace_x, double* trace_y, double* trace_xa, double* trace_ya,
                 int32_t* trace_cg, double* trace_step, const or_original* orig) {
    int64_t n = Q->nrows, m = A->nrows;
    double* x = alloc(n);
    double* y = alloc(m);
    double* xn = alloc(n);
    double* yn = alloc(m);
    double* xa = alloc(n);  /* running averages */
    double* ya = alloc(m);
    double* x_anc = alloc(n);  /* epoch anchor z^{n,0} */
    double* y_anc = alloc(m);
    double* g = alloc(n);
    double* Aty = alloc(n);
    double* Ax = alloc(m);
    double* Axn = alloc(m);
    double* xm = alloc(n);  /* work space of kkt_at */
    double* ym = alloc(m);
    double kk[8], ka[8];

    double normA = or_opnorm(A, s->power_iters);
    double eta = s->eta_factor / (normA > 0.0 ? normA : 1.0);
    double omega = s->pw_init;
    double tau = eta / omega, sigma = eta * omega;

    for (int64_t j = 0; j < n; ++j) x[j] = x0 ? x0[j] : 0.0;
    for (int64_t i = 0; i < m; ++i) y[i] = y0 ? (y0[i] > 0.0 ? y0[i] : 0.0) : 0.0;

    int64_t k = 0, k_total = 0, cg_total = 0, restarts = 0, rejections = 0;
    double eps = 0.0;
    double K_anchor, K_prev = INFINITY;
    int32_t status = OR_ITER_LIMIT, ret_avg = 0;

    kkt_at(Q, A, b, c, orig, x, y, kk, xm, ym);
    K_anchor = kk[3];
    memcpy(x_anc, x, sizeof(double) * n);
    memcpy(y_anc, y, sizeof(double) * m);
    memcpy(xa, x, sizeof(double) * n);
    memcpy(ya, y, sizeof(double) * m);

    for (;;) {
        /* relKKT of the current iterate: termination and the CG tolerance */
        kkt_at(Q, A, b, c, orig, x, y, kk, xm, ym);
        if (!isfinite(kk[3])) {
            status = OR_NUMERICAL;
            memcpy(x, x_anc, sizeof(double) * n);
            memcpy(y, y_anc, sizeof(double) * m);
            kkt_at(Q, A, b, c, orig, x, y, kk, xm, ym);
            break;
        }
        if (kk[3] <= s->tol) { status = OR_OPTIMAL; break; }

        if (k > 0 && k % s->eval_period == 0) {
            kkt_at(Q, A, b, c, orig, xa, ya, ka, xm, ym);
            if (ka[3] <= s->tol) {
                status = OR_OPTIMAL;
                memcpy(x, xa, sizeof(double) * n);
                memcpy(y, ya, sizeof(double) * m);
                memcpy(kk, ka, sizeof kk);
                ret_avg = 1;
                break;
            }
            int use_avg = (s->restart_to == 1) || (ka[3] < kk[3]);
            double K_c = use_avg ? ka[3] : kk[3];
            int32_t why = or_restart_decision(K_c, K_anchor, K_prev, k, k_total, s->beta_suf, s->beta_nec,
                                              s->beta_art);
            K_prev = K_c;
            if (why) {
                const double* xc = use_avg ? xa : x;
                const double* yc = use_avg ? ya : y;
                double dx = dist2(n, xc, x_anc), dy = dist2(m, yc, y_anc);
                if (s->pw_theta > 0.0) omega = or_primal_weight(omega, dx, dy, s->pw_theta);
                tau = eta / omega;
                sigma = eta * omega;
                if (use_avg) {
                    memcpy(x, xa, sizeof(double) * n);
                    memcpy(y, ya, sizeof(double) * m);
                    memcpy(kk, ka, sizeof kk);
                }
                memcpy(x_anc, x, sizeof(double) * n);
                memcpy(y_anc, y, sizeof(double) * m);
                memcpy(xa, x, sizeof(double) * n);
                memcpy(ya, y, sizeof(double) * m);
                K_anchor = K_c;
                K_prev = INFINITY;
                k = 0;
                eps = 0.0;
                restarts++;
            }
        }

        if (k_total >= s->max_iters) {
            if (k > 0) {
                kkt_at(Q, A, b, c, orig, xa, ya, ka, xm, ym);
                if (ka[3] < kk[3]) {
                    memcpy(x, xa, sizeof(double) * n);
                    memcpy(y, ya, sizeof(double) * m);
                    memcpy(kk, ka, sizeof kk);
                    ret_avg = 1;
                }
            }
            status = kk[3] <= s->tol ? OR_OPTIMAL : OR_ITER_LIMIT;
            break;
        }

        eps += s->cg_eps_factor * kk[3];

        /* g = Q x^k + A'y^k + c: the CG's starting residual is -g */
        or_matvec(Q, x, g);
        or_matvec_t(A, y, Aty);
        for (int64_t j = 0; j < n; ++j) g[j] += Aty[j] + c[j];
        or_matvec(A, x, Ax);
        int32_t steps = 0, attempts = 0;
        double eta_used = eta, eta_bar = INFINITY;
        for (;;) {
            /* primal step: CG on (Q + I/tau) x = x^k/tau - c - A'y^k from x^k */
            memcpy(xn, x, sizeof(double) * n);
            steps += or_cg(Q, tau, g, xn, eps, s->max_cg, s->cg_rule);
            /* dual step at the extrapolated point 2x^{k+1} - x^k */
            or_matvec(A, xn, Axn);
            for (int64_t i = 0; i < m; ++i) yn[i] = fmax(0.0, y[i] + sigma * (2.0 * Axn[i] - Ax[i] - b[i]));
            attempts++;
            if (s->step_rule == 0) break;
            /* adaptive step (Sec. 4): accept when eta <= eta_bar; the next
             * attempt or iteration uses eta' either way (64 attempts at most,
             * the last accepted: a bound never reached in the tests) */
            eta_used = eta;
            eta_bar = or_step_limit(Q, A, x, xn, y, yn, omega);
            int accept = eta <= eta_bar || attempts >= 64;
            eta = or_next_step(eta, eta_bar, k_total + 1);
            tau = eta / omega;
            sigma = eta * omega;
            if (accept) break;
            rejections++;
        }
        cg_total += steps;

        /* running averages, weight 1/(k+1) */
        double w = 1.0 / (double)(k + 1);
        for (int64_t j = 0; j < n; ++j) xa[j] += w * (xn[j] - xa[j]);
        for (int64_t i = 0; i < m; ++i) ya[i] += w * (yn[i] - ya[i]);

        memcpy(x, xn, sizeof(double) * n);
        memcpy(y, yn, sizeof(double) * m);
        if (k_total < trace_len) {
            memcpy(trace_x + k_total * n, x, sizeof(double) * n);
            memcpy(trace_y + k_total * m, y, sizeof(double) * m);
            memcpy(trace_xa + k_total * n, xa, sizeof(double) * n);
            memcpy(trace_ya + k_total * m, ya, sizeof(double) * m);
            trace_cg[k_total] = steps;
            if (trace_step) {
                trace_step[3 * k_total] = eta_used;
                trace_step[3 * k_total + 1] = eta_bar;
                trace_step[3 * k_total + 2] = (double)attempts;
            }
        }
        k++;
        k_total++;
    }

    memcpy(x_out, x, sizeof(double) * n);
    memcpy(y_out, y, sizeof(double) * m);
    info[0] = status;
    info[1] = (double)k_total;
    info[2] = (double)cg_total;
    info[3] = (double)restarts;
    info[4] = ret_avg;
    for (int t = 0; t < 4; ++t) info[5 + t] = kk[t];
    info[9] = kk[4];
    info[10] = kk[5];
    info[11] = normA;
    info[12] = (double)rejections;
    free(x); free(y); free(xn); free(yn); free(xa); free(ya); free(x_anc); free(y_anc);
    free(g); free(Aty); free(Ax); free(Axn); free(xm); free(ym);
    return status;
}

int32_t or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
