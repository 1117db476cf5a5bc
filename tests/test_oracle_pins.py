"""Pins of the FP64 CPU oracle against results fixed by the paper or by
mathematics (closed forms, brute force, library routines), never against the
oracle itself.  CPU only."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import oracle as O
from paper_2405_16160_amd import instances as I

SQ2 = math.sqrt(2.0)


def _qp_dense(Q, c, A, b):
    return I.QP(I.CSR.from_scipy(sp.csr_matrix(np.atleast_2d(Q))), I.CSR.from_scipy(sp.csr_matrix(np.atleast_2d(A))),
                np.asarray(b, float), np.asarray(c, float))


def example_w():
    """Worked example W: Q = diag(2,1), c = (-2,-1), A = [1 1], b = 1.
    Optimum x* = (2/3, 1/3), y* = 2/3, objective -7/6 (KKT by hand)."""
    return _qp_dense(np.diag([2.0, 1.0]), [-2.0, -1.0], [[1.0, 1.0]], [1.0])


# --------------------------------------------------------------- relKKT

def test_relkkt_worked_example():
    """relKKT (Sec. 4, progress metric) on W at three points, by hand:
    (0,0): r_p = 0, r_d = 2/(1+2) = 2/3, r_g = 0;
    ((1,1),0): Ax - b = 1 -> r_p = 1/(1+2) = 1/3, Qx + c = 0, gap 3 - 3 + 0 = 0;
    (x*, y*): all zero; objectives -7/6 (primal and dual)."""
    qp = example_w()
    k = O.kkt(qp, [0, 0], [0])
    assert k["r_primal"] == 0.0 and k["r_gap"] == 0.0
    assert k["r_dual"] == pytest.approx(2 / 3, abs=1e-15) and k["rel_kkt"] == pytest.approx(2 / 3, abs=1e-15)
    k = O.kkt(qp, [1, 1], [0])
    assert k["r_primal"] == pytest.approx(1 / 3, abs=1e-15)
    assert k["r_dual"] == 0.0 and k["r_gap"] == 0.0
    k = O.kkt(qp, [2 / 3, 1 / 3], [2 / 3])
    assert k["rel_kkt"] < 1e-15
    assert k["primal_obj"] == pytest.approx(-7 / 6, abs=1e-15)
    assert k["dual_obj"] == pytest.approx(-7 / 6, abs=1e-15)


def test_relkkt_dual_gap_signs():
    """Gap numerator x'Qx + c'x + b'y: a point with stationarity but the wrong
    dual value must show a gap (guards a sign slip in the gap term)."""
    qp = example_w()
    # x*, but y = 0 is not stationary; y = 1 stationary? Qx + c + A'y = (-2/3+1, -2/3+1) != 0
    k = O.kkt(qp, [2 / 3, 1 / 3], [1.0])
    # by hand: x'Qx = 1, c'x = -5/3, b'y = 1 -> gap = 1/3; denominators 1 + max(7/6, 3/2)
    assert k["r_gap"] == pytest.approx((1 / 3) / (1 + 1.5), abs=1e-15)
    # dual residual (1/3, 1/3) / (1 + max(4/3, 1, 2))
    assert k["r_dual"] == pytest.approx((1 / 3) / 3.0, abs=1e-15)


# --------------------------------------------------- first steps of Alg. 1

def _w_settings(**kw):
    s = O.Settings(tol=1e-14, max_iters=2, eval_period=10_000, power_iters=50, **kw)
    return s


def test_first_two_iterations_exact_cg():
    """Alg. 1 on W from (0,0) with sigma = tau = 1/(2||A||) = 1/(2 sqrt 2)
    (Thm 2) and CG run to its finite termination (2 steps, tolerance 0):
    x1 = (2, 1) ./ (diag(Q) + 1/tau) = (sqrt2 - 1, 1/(1 + 2 sqrt2)),
    y1 = sigma (A (2 x1) - b), then x2 = (x1/tau - c - A'y1) ./ (diag(Q) + 1/tau),
    y2 = y1 + sigma (A(2 x2 - x1) - b).  Closed forms derived by hand."""
    qp = example_w()
    r = O.solve(qp, _w_settings(max_cg=2, cg_eps_factor=0.0), trace_len=2)
    assert r.norm_A == pytest.approx(SQ2, rel=1e-14)
    tau = sigma = 1 / (2 * SQ2)
    d = np.array([2 + 1 / tau, 1 + 1 / tau])
    x1 = np.array([SQ2 - 1, 1 / (1 + 2 * SQ2)])
    assert np.allclose(x1, np.array([2.0, 1.0]) / d, atol=1e-15)
    y1 = sigma * (2 * x1.sum() - 1)
    x2 = (x1 / tau - np.array([-2.0, -1.0]) - y1) / d
    y2 = y1 + sigma * ((2 * x2 - x1).sum() - 1)
    assert np.allclose(r.trace_x[0], x1, atol=1e-14)
    assert r.trace_y[0][0] == pytest.approx(y1, abs=1e-14)
    assert np.allclose(r.trace_x[1], x2, atol=1e-14)
    assert r.trace_y[1][0] == pytest.approx(y2, abs=1e-14)
    # decimal values of the same closed forms
    assert np.allclose(r.trace_x[0], [0.41421356, 0.26120387], atol=1e-8)
    assert r.trace_y[0][0] == pytest.approx(0.12403886, abs=1e-8)
    assert np.allclose(r.trace_x[1], [0.63116496, 0.42178085], atol=2e-8)
    assert r.trace_y[1][0] == pytest.approx(0.27623447, abs=1e-8)
    # averages are the uniform means of the iterates of the epoch
    assert np.allclose(r.trace_xa[0], x1, atol=1e-15)
    assert np.allclose(r.trace_xa[1], (x1 + x2) / 2, atol=1e-15)
    assert r.trace_ya[1][0] == pytest.approx((y1 + y2) / 2, abs=1e-15)
    assert list(r.trace_cg) == [2, 2]


def test_first_iteration_cg_capped_at_one_step():
    """PDHCG-fixed with N = 1 on W: one CG step from x0 = 0 along r0 = (2,1),
    alpha = |r0|^2 / r0'(Q + I/tau) r0 = 5 / (9 + 10 sqrt2), x1 = alpha (2,1),
    y1 = sigma (2 (x1_1 + x1_2) - 1)."""
    qp = example_w()
    r = O.solve(qp, _w_settings(max_cg=1, cg_rule=1), trace_len=1)
    alpha = 5 / (9 + 10 * SQ2)
    assert alpha == pytest.approx(0.21605612, abs=1e-8)
    x1 = alpha * np.array([2.0, 1.0])
    y1 = (2 * x1.sum() - 1) / (2 * SQ2)
    assert y1 == pytest.approx(0.10477085, abs=1e-8)
    assert np.allclose(r.trace_x[0], x1, atol=1e-15)
    assert r.trace_y[0][0] == pytest.approx(y1, abs=1e-15)


def test_worked_example_converges():
    r = O.solve(example_w(), O.Settings(tol=1e-10))
    assert r.status == O.OPTIMAL
    assert np.allclose(r.x, [2 / 3, 1 / 3], atol=1e-8)
    assert r.y[0] == pytest.approx(2 / 3, abs=1e-8)


# ------------------------------------------------------------ primitives

def test_matvec_against_scipy():
    qp = I.random_qp(300, 150, q_density=0.03, a_density=0.03, family=21)
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal(300), rng.standard_normal(150)
    A = qp.A.to_scipy()
    assert np.allclose(O.matvec(qp.A, x), A @ x, rtol=1e-13, atol=1e-13)
    assert np.allclose(O.matvec_t(qp.A, y), A.T @ y, rtol=1e-13, atol=1e-13)


def test_opnorm_matches_svd():
    rng = np.random.default_rng(1)
    for shape in [(30, 20), (7, 40), (50, 50)]:
        M = rng.standard_normal(shape)
        exact = np.linalg.norm(M, 2)
        est = O.opnorm(I.CSR.from_scipy(sp.csr_matrix(M)), 300)
        assert est == pytest.approx(exact, rel=1e-6)
        assert est <= exact * (1 + 1e-12)   # power iteration never overshoots


def test_opnorm_of_difference_row():
    """A = [1, -1]: the all-ones start would be in the null space; the fixed
    non-uniform start still finds ||A|| = sqrt 2."""
    est = O.opnorm(I.CSR.from_scipy(sp.csr_matrix(np.array([[1.0, -1.0]]))), 20)
    assert est == pytest.approx(SQ2, rel=1e-12)


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    return G.T @ G / n + 0.05 * np.eye(n)


def test_cg_to_convergence_matches_dense_solve():
    """CG on (Q + I/tau) x = x0/tau - g' (Sec. 2): with tolerance 0 and n steps
    it reaches the dense solution (finite termination in exact arithmetic)."""
    n, tau = 40, 0.3
    Qd = _spd(n, 2)
    Q = I.CSR.from_scipy(sp.csr_matrix(Qd))
    rng = np.random.default_rng(3)
    x0 = rng.standard_normal(n)
    g = rng.standard_normal(n)          # = Q x0 + A'y + c
    xs, steps = O.cg(Q, tau, g, x0, 0.0, 3 * n)
    M = Qd + np.eye(n) / tau
    exact = x0 + np.linalg.solve(M, -g)
    assert np.linalg.norm(xs - exact) / np.linalg.norm(exact) < 1e-12
    assert steps <= 3 * n


def test_cg_one_step_closed_form():
    n, tau = 25, 0.7
    Qd = _spd(n, 4)
    Q = I.CSR.from_scipy(sp.csr_matrix(Qd))
    rng = np.random.default_rng(5)
    x0, g = rng.standard_normal(n), rng.standard_normal(n)
    x1, steps = O.cg(Q, tau, g, x0, 1e300, 50)   # huge tolerance: exactly one step
    r0 = -g
    M = Qd + np.eye(n) / tau
    alpha = (r0 @ r0) / (r0 @ M @ r0)
    assert steps == 1
    assert np.allclose(x1, x0 + alpha * r0, rtol=1e-14, atol=1e-14)


def test_cg_stop_rule_and_error_bound():
    """The stop test certifies ||x_l - x*|| <= tau ||r_l|| <= eps, and the
    textbook CG bound ||e_l||_M <= 2 ((sqrt k - 1)/(sqrt k + 1))^l ||e_0||_M
    holds at every step (Sec. 2 quotes the same rate)."""
    n, tau = 60, 0.5
    Qd = _spd(n, 6) * 10
    Q = I.CSR.from_scipy(sp.csr_matrix(Qd))
    M = Qd + np.eye(n) / tau
    rng = np.random.default_rng(7)
    x0, g = rng.standard_normal(n), rng.standard_normal(n)
    exact = x0 + np.linalg.solve(M, -g)
    eps = 1e-3
    x, steps = O.cg(Q, tau, g, x0, eps, 500)
    assert np.linalg.norm(x - exact) <= eps
    r = -g - M @ (x - x0)
    assert tau * np.linalg.norm(r) <= eps * (1 + 1e-12)
    if steps > 1:
        xp, sp_ = O.cg(Q, tau, g, x0, 0.0, steps - 1)
        rp = -g - M @ (xp - x0)
        assert tau * np.linalg.norm(rp) > eps
    ev = np.linalg.eigvalsh(M)
    kap = ev[-1] / ev[0]
    rate = (math.sqrt(kap) - 1) / (math.sqrt(kap) + 1)
    e0 = x0 - exact
    nM = lambda e: math.sqrt(e @ M @ e)
    for l in range(1, 15):
        xl, _ = O.cg(Q, tau, g, x0, 0.0, l)
        assert nM(xl - exact) <= 2 * rate ** l * nM(e0) * (1 + 1e-9) + 1e-13


# ----------------------------------------------- restart and primal weight

def _load_restart_table():
    rows = []
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "restart_table.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            parts = line.split()
            K_c, K_anchor, K_prev = float(parts[0]), float(parts[1]), float(parts[2])
            k, k_total, expect = int(parts[3]), int(parts[4]), int(parts[5])
            rows.append((K_c, K_anchor, K_prev, k, k_total, expect))
    return rows


@pytest.mark.parametrize("row", _load_restart_table())
def test_restart_decision_table(row):
    K_c, K_anchor, K_prev, k, k_total, expect = row
    assert O.restart_decision(K_c, K_anchor, K_prev, k, k_total) == expect


def test_primal_weight_worked_value():
    """omega' = exp(theta log(dy/dx) + (1-theta) log omega) (Sec. 4): with
    omega = 1, dx = 1, dy = e^5, theta = 0.2 this is e^1."""
    assert O.primal_weight(1.0, 1.0, math.exp(5.0), 0.2) == pytest.approx(math.e, rel=1e-14)
    # omega = 4, dy/dx = 1/4, theta = 0.5 -> exp(0.5 log(1/4) + 0.5 log 4) = 1
    assert O.primal_weight(4.0, 2.0, 0.5, 0.5) == pytest.approx(1.0, rel=1e-14)
    # no update when a movement is (numerically) zero
    assert O.primal_weight(3.0, 0.0, 1.0, 0.2) == 3.0
    assert O.primal_weight(3.0, 1.0, 1e-12, 0.2) == 3.0


# ------------------------------------------------------- whole solves

def brute_force_active_set(Q, c, A, b):
    """Enumerate active sets S (|S| <= n, A_S full row rank); solve the KKT
    system [[Q, A_S'], [A_S, 0]] [x; y_S] = [-c; b_S]; keep primal-feasible
    points with y_S >= 0; return the one of least objective."""
    n, m = Q.shape[0], A.shape[0]
    best = None
    tolb = 1e-9 * (1 + np.abs(b).max())
    for size in range(0, min(n, m) + 1):
        for S in itertools.combinations(range(m), size):
            S = list(S)
            AS = A[S]
            if size and np.linalg.matrix_rank(AS) < size:
                continue
            K = np.block([[Q, AS.T], [AS, np.zeros((size, size))]])
            rhs = np.concatenate([-c, b[S]])
            try:
                sol = np.linalg.solve(K, rhs)
            except np.linalg.LinAlgError:
                continue
            x, yS = sol[:n], sol[n:]
            if np.any(A @ x > b + tolb) or np.any(yS < -1e-12):
                continue
            f = 0.5 * x @ Q @ x + c @ x
            if best is None or f < best[0] - 1e-12:
                y = np.zeros(m)
                y[S] = yS
                best = (f, x, y)
    return best


@pytest.mark.parametrize("n,m,inst", [(2, 3, 0), (3, 5, 1), (4, 6, 2), (5, 8, 3), (6, 10, 4), (8, 12, 5)])
def test_whole_solve_against_brute_force(n, m, inst):
    qp = I.tiny_qp(n, m, instance=inst)
    Q = qp.Q.to_scipy().toarray()
    A = qp.A.to_scipy().toarray()
    f, xs, ys = brute_force_active_set(Q, qp.c, A, qp.b)
    r = O.solve(qp, O.Settings(tol=1e-11, max_iters=400_000))
    assert r.status == O.OPTIMAL, (r.status, r.iters, r.rel_kkt)
    assert np.linalg.norm(r.x - xs) <= 1e-7 * max(1.0, np.linalg.norm(xs))
    assert r.primal_obj == pytest.approx(f, rel=1e-8, abs=1e-8)
    assert np.all(r.y >= 0)


def test_inactive_constraints_closed_form():
    """b = A(-Q^{-1} c) + U[0.1, 1]: no constraint is active, so x* = -Q^{-1} c
    and y* = 0 (Cholesky of the tiny-case Q)."""
    base = I.random_qp(family=31)
    Qd = base.Q.to_scipy().toarray()
    L = np.linalg.cholesky(Qd)
    xs = -np.linalg.solve(L.T, np.linalg.solve(L, base.c))
    rng = np.random.default_rng(32)
    b = base.A.to_scipy() @ xs + rng.uniform(0.1, 1.0, base.m)
    qp = I.QP(base.Q, base.A, b, base.c)
    r = O.solve(qp, O.Settings(tol=1e-9))
    assert r.status == O.OPTIMAL
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 1e-6
    assert np.abs(r.y).max() < 1e-6


def test_all_rows_active_kkt_solve():
    """Every row active with y* > 0 (manufactured with active fraction 1): x*
    and y* come from the KKT system; y* is unique since A has full row rank."""
    qp = I.manufactured(n=120, m=40, q_density=0.1, a_density=0.1, active_frac=1.0, family=33)
    r = O.solve(qp, O.Settings(tol=1e-10))
    assert r.status == O.OPTIMAL
    assert np.linalg.norm(r.x - qp.x_star) / np.linalg.norm(qp.x_star) < 1e-6
    assert np.linalg.norm(r.y - qp.y_star) / np.linalg.norm(qp.y_star) < 1e-5


def test_manufactured_solution_tiny_case_size():
    qp = I.manufactured()
    r = O.solve(qp, O.Settings(tol=1e-9))
    assert r.status == O.OPTIMAL
    assert np.linalg.norm(r.x - qp.x_star) / np.linalg.norm(qp.x_star) < 1e-6
    f = 0.5 * qp.x_star @ (qp.Q.to_scipy() @ qp.x_star) + qp.c @ qp.x_star
    assert abs(r.primal_obj - f) / (1 + abs(f)) < 1e-8


def test_unconstrained_is_proximal_point():
    """m = 0: PDHCG reduces to proximal point iterations; x* = -Q^{-1} c."""
    qp = I.unconstrained(150)
    xs = -np.linalg.solve(qp.Q.to_scipy().toarray(), qp.c)
    r = O.solve(qp, O.Settings(tol=1e-10))
    assert r.status == O.OPTIMAL
    assert np.linalg.norm(r.x - xs) / np.linalg.norm(xs) < 1e-8


def test_invariants_along_iterations():
    """y >= 0 after every projection; the averages are the uniform means of
    the iterates since the last restart (checked over the first epoch)."""
    qp = I.random_qp(family=34)
    T = 60
    r = O.solve(qp, O.Settings(tol=1e-12, max_iters=T), trace_len=T)
    assert np.all(r.trace_y >= 0)
    for k in (0, 9, 59):
        assert np.allclose(r.trace_xa[k], r.trace_x[: k + 1].mean(axis=0), atol=1e-12)
        assert np.allclose(r.trace_ya[k], r.trace_y[: k + 1].mean(axis=0), atol=1e-12)
    assert np.all(r.trace_cg >= 1)


def test_cg_steps_bounded_and_anchor_decreases():
    """Qualitative (Prop. 1, Thm 2): CG steps per iteration stay bounded well
    below the cap, and the solve converges on the tiny case."""
    qp = I.random_qp()
    r = O.solve(qp, O.Settings(tol=1e-6))
    assert r.status == O.OPTIMAL
    assert r.cg_steps / r.iters < 30


def test_failure_modes():
    qp = example_w()
    # NaN in c -> NUMERICAL_ERROR
    bad = I.QP(qp.Q, qp.A, qp.b, np.array([np.nan, 1.0]))
    assert O.solve(bad).status == O.NUMERICAL_ERROR
    # infeasible pair x1 <= -1, -x1 <= -1 -> iteration limit
    inf = _qp_dense(np.eye(1), [0.0], [[1.0], [-1.0]], [-1.0, -1.0])
    r = O.solve(inf, O.Settings(max_iters=2000))
    assert r.status == O.ITER_LIMIT
    # iteration cap
    r = O.solve(I.random_qp(), O.Settings(tol=1e-12, max_iters=10))
    assert r.status == O.ITER_LIMIT and r.iters == 10


def test_warm_start_resume_and_negative_y0():
    qp = I.random_qp(family=35)
    r1 = O.solve(qp, O.Settings(tol=1e-7, max_iters=200))
    assert r1.status == O.ITER_LIMIT
    r2 = O.solve(qp, O.Settings(tol=1e-7), x0=r1.x, y0=r1.y)
    assert r2.status == O.OPTIMAL
    ref = O.solve(qp, O.Settings(tol=1e-9))
    assert np.linalg.norm(r2.x - ref.x) / np.linalg.norm(ref.x) < 1e-4
    # a negative warm-start dual is projected onto y >= 0 before the first step
    y0 = -np.ones(qp.m)
    r3 = O.solve(qp, O.Settings(tol=1e-12, max_iters=1), y0=y0, trace_len=1)
    r4 = O.solve(qp, O.Settings(tol=1e-12, max_iters=1), y0=np.zeros(qp.m), trace_len=1)
    assert np.array_equal(r3.trace_x[0], r4.trace_x[0])
