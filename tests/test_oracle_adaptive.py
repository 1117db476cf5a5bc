"""Pins of the oracle's adaptive step size (Sec. 4, "Adaptive step-size": the
PDLP step rule with the QP-specific limit
eta <= ||z' - z||_w^2 / (2 |dx'A'dy| + dx'Q dx)) against values derived by
hand on the worked example W, closed forms of the step update, dense solves of
the proximal subproblem (a library routine), invariants along a solve, and the
exact optima of whole solves.  CPU only.  The hand values below come from the
closed forms of the first trial step on W (x1 = (sqrt2 - 1, 1/(1 + 2 sqrt2)),
y1 = sigma (2 (x1_1 + x1_2) - 1) at sigma = tau = 1/(2 sqrt2)) and are listed,
with their derivation, in tests/golden/adaptive_step_W.txt."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_16160_amd import instances as I
from test_oracle_pins import SQ2, example_w, _qp_dense, _w_settings

# the first trial step on W from (0, 0) at eta = 0.5/sqrt2 (tests/golden/adaptive_step_W.txt)
X1 = np.array([SQ2 - 1.0, 1.0 / (1.0 + 2.0 * SQ2)])
Y1 = 0.1240388594792434
ETA_BAR_1 = 0.4407895889587272        # (|dx|^2 + dy^2) / (2 dy (dx_1 + dx_2) + 2 dx_1^2 + dx_2^2)
ETA_BAR_1_W2 = 0.8417151380390061     # the same with omega = 2: (2 |dx|^2 + dy^2 / 2) / den
ETA_BAR_NEG = 0.4506850869440022      # y = 1 -> 0.5: the bilinear term -0.5 (dx_1 + dx_2) by magnitude
RED, GROW = 1.0 - 2.0 ** -0.3, 1.0 + 2.0 ** -0.6   # the update factors at t = 1
REJ_ETA_BAR = 1.8180652825233083      # trial at eta = 4/sqrt2 from (0, 0): x' = (2, 1)/(diag Q + 1/tau), y' = tau (2 sum x' - 1)
REJ_ETA_1 = 0.3413374000616747        # RED * REJ_ETA_BAR (smaller than GROW * 4/sqrt2)
REJ_ETA_BAR_2 = 0.44825557519401565   # trial at REJ_ETA_1: accepted


def test_step_limit_worked_example():
    qp = example_w()
    z, zy = np.zeros(2), np.zeros(1)
    assert O.step_limit(qp, z, X1, zy, [Y1]) == pytest.approx(ETA_BAR_1, rel=1e-14)
    assert O.step_limit(qp, z, X1, zy, [Y1], omega=2.0) == pytest.approx(ETA_BAR_1_W2, rel=1e-14)
    # a dual step that decreases y: the bilinear term counts by its magnitude
    assert O.step_limit(qp, z, X1, [1.0], [0.5]) == pytest.approx(ETA_BAR_NEG, rel=1e-14)
    # no movement: no limit
    assert math.isinf(O.step_limit(qp, X1, X1, [Y1], [Y1]))
    # only the Q term left (dy = 0): omega |dx|^2 / dx'Q dx
    assert O.step_limit(qp, z, np.array([1.0, 0.0]), zy, zy) == pytest.approx(0.5, rel=1e-15)


def test_next_step_closed_form():
    # t = 1: min((1 - 2^-0.3) eta_bar, (1 + 2^-0.6) eta)
    assert O.next_step(1.0, 10.0, 1) == pytest.approx(GROW, rel=1e-15)
    assert O.next_step(1.0, 1.0, 1) == pytest.approx(RED, rel=1e-15)
    assert RED == pytest.approx(0.18774760364376442, rel=1e-15) and GROW == pytest.approx(1.659753955386447, rel=1e-15)
    # large t: the limit factor tends to 1 and the growth factor to 1
    t = 10 ** 8
    assert O.next_step(1.0, 0.5, t) == pytest.approx(0.5 * (1 - (t + 1.0) ** -0.3), rel=1e-15)
    assert O.next_step(0.5, math.inf, t) == pytest.approx(0.5 * (1 + (t + 1.0) ** -0.6), rel=1e-15)


def _solve_w(**kw):
    return O.solve(example_w(), _w_settings(max_cg=2, cg_eps_factor=0.0, step_rule=1, **kw), trace_len=2)


def test_first_adaptive_iteration_on_w_is_accepted():
    """At eta0 = 0.5/sqrt2 the first trial satisfies eta0 <= eta_bar: it is
    the constant rule's x1, y1, and the next step is RED * eta_bar; the second
    iteration takes the proximal step with tau = sigma = that step (dense
    solve of (Q + I/tau) x = x1/tau - c - A'y1)."""
    r = _solve_w()
    assert r.rejections == 0
    eta0 = 0.5 / SQ2
    assert np.allclose(r.trace_x[0], X1, atol=1e-15) and r.trace_y[0][0] == pytest.approx(Y1, abs=1e-15)
    assert r.trace_step[0][0] == pytest.approx(eta0, rel=1e-15)
    assert r.trace_step[0][1] == pytest.approx(ETA_BAR_1, rel=1e-13)
    assert r.trace_step[0][2] == 1
    eta1 = RED * ETA_BAR_1
    assert eta1 < GROW * eta0
    assert r.trace_step[1][0] == pytest.approx(eta1, rel=1e-13)
    tau = sig = eta1
    Q, c, A, b = np.diag([2.0, 1.0]), np.array([-2.0, -1.0]), np.array([[1.0, 1.0]]), np.array([1.0])
    x2 = np.linalg.solve(Q + np.eye(2) / tau, X1 / tau - c - A.T @ [Y1])
    y2 = max(0.0, Y1 + sig * ((A @ (2 * x2 - X1))[0] - b[0]))
    assert np.allclose(r.trace_x[1], x2, atol=1e-13)
    assert r.trace_y[1][0] == pytest.approx(y2, abs=1e-13)


def test_rejected_trial_on_w():
    """From eta0 = 4/sqrt2 the first trial violates the limit (eta0 > eta_bar =
    1.818...): it is rejected, eta becomes RED * eta_bar, and the repeated
    trial from (0, 0) (dense solve at tau = sigma = that eta) is accepted."""
    r = _solve_w(eta_factor=4.0)
    assert r.rejections == 1
    assert r.trace_step[0][2] == 2
    assert r.trace_step[0][0] == pytest.approx(REJ_ETA_1, rel=1e-12)
    assert r.trace_step[0][1] == pytest.approx(REJ_ETA_BAR_2, rel=1e-12)
    assert RED * REJ_ETA_BAR == pytest.approx(REJ_ETA_1, rel=1e-14)
    tau = REJ_ETA_1
    x1 = np.array([2.0, 1.0]) / (np.array([2.0, 1.0]) + 1.0 / tau)
    y1 = tau * (2 * x1.sum() - 1.0)
    assert np.allclose(r.trace_x[0], x1, atol=1e-14)
    assert r.trace_y[0][0] == pytest.approx(y1, abs=1e-14)
    # the CG steps of the rejected trial count too (2 per trial on W)
    assert r.trace_cg[0] == 4


def test_invariants_along_an_adaptive_solve():
    """Every accepted trial satisfies eta <= eta_bar; the step grows by at most
    the factor 1 + (t+1)^-0.6 per iteration; the solve reaches the tolerance
    and the same x* as the constant-step solve (x* is unique)."""
    qp = I.random_qp(n=300, m=150, r_rows=150, q_density=0.03, a_density=0.03, family=1, instance=7)
    r = O.solve(qp, O.Settings(tol=1e-9, step_rule=1), trace_len=400)
    assert r.status == O.OPTIMAL
    ts = r.trace_step
    assert np.all((ts[:, 0] <= ts[:, 1]) | (ts[:, 2] >= 64))
    t = np.arange(1, len(ts))
    assert np.all(ts[1:, 0] <= (1 + (t + 1.0) ** -0.6) * ts[:-1, 0] * (1 + 1e-15))
    ref = O.solve(qp, O.Settings(tol=1e-10))
    assert np.linalg.norm(r.x - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def _brute_force(qp):
    """Exact optimum by active-set enumeration (n <= 8, m <= 12)."""
    import itertools
    Q, A = qp.Q.to_scipy().toarray(), qp.A.to_scipy().toarray()
    b, c = qp.b, qp.c
    n, m = Q.shape[0], A.shape[0]
    best = None
    for k in range(0, min(n, m) + 1):
        for S in itertools.combinations(range(m), k):
            S = list(S)
            K = np.block([[Q, A[S].T], [A[S], np.zeros((k, k))]]) if k else Q
            rhs = np.concatenate([-c, b[S]]) if k else -c
            try:
                sol = np.linalg.solve(K, rhs)
            except np.linalg.LinAlgError:
                continue
            x, yS = sol[:n], sol[n:]
            if np.all(A @ x <= b + 1e-9 * (1 + np.abs(b).max())) and np.all(yS >= -1e-12):
                f = 0.5 * x @ Q @ x + c @ x
                if best is None or f < best[0]:
                    best = (f, x)
    return best[1]


@pytest.mark.parametrize("inst", range(4))
def test_adaptive_whole_solve_reaches_the_exact_optimum(inst):
    qp = I.tiny_qp(6, 10, instance=inst)
    r = O.solve(qp, O.Settings(tol=1e-11, step_rule=1, max_iters=400_000))
    assert r.status == O.OPTIMAL
    xs = _brute_force(qp)
    assert np.linalg.norm(r.x - xs) <= 1e-7 * max(1.0, np.linalg.norm(xs))


def test_adaptive_manufactured_optimum_and_unconstrained():
    qp = I.manufactured(n=300, m=150, q_density=0.03, a_density=0.03, instance=4)
    r = O.solve(qp, O.Settings(tol=1e-10, step_rule=1))
    assert r.status == O.OPTIMAL
    assert np.linalg.norm(r.x - qp.x_star) <= 1e-6 * np.linalg.norm(qp.x_star)
    # m = 0: the limit is omega |dx|^2 / dx'Q dx; the solve reaches -Q^-1 c
    qu = I.unconstrained(80)
    ru = O.solve(qu, O.Settings(tol=1e-11, step_rule=1))
    xs = -np.linalg.solve(qu.Q.to_scipy().toarray(), qu.c)
    assert ru.status == O.OPTIMAL and np.linalg.norm(ru.x - xs) <= 1e-8 * np.linalg.norm(xs)
