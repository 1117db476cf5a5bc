"""Pins of the oracle's diagonal preconditioning (Ruiz + Pock-Chambolle on
K = [[Q, A'], [A, 0]], Sec. 4, "Preprocessing") against hand-derived closed forms, the
defining property of Ruiz equilibration and the invariance of the solution
under the rescaling, and a check that each pin set catches planted mistakes.
CPU only."""
import math
import pathlib
import types

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import oracle as O
from oracle import precondition as P
from paper_2405_16160_amd import instances as I


def _qp(Q, A, b, c):
    return I.QP(I.CSR.from_scipy(sp.csr_matrix(np.atleast_2d(np.asarray(Q, float)))),
                I.CSR.from_scipy(sp.csr_matrix(np.atleast_2d(np.asarray(A, float)))),
                np.asarray(b, float), np.asarray(c, float))


def test_one_by_one_closed_form():
    # K = [[4, 1], [1, 0]].  Ruiz step 1 divides index 0 by sqrt(4) and leaves
    # index 1 (row max 1): K -> [[1, 1/2], [1/2, 0]].  From then on the row max
    # of index 0 stays 1 and the off-diagonal a_k obeys a_{k+1} = sqrt(a_k), so
    # after 10 steps a = 2^(-2^-9), d2 = 1/2, d1 = 2^(1 - 2^-9).  The
    # Pock-Chambolle step then divides index 0 by sqrt(1 + a) and index 1 by
    # sqrt(a).
    qp = _qp([[4.0]], [[1.0]], [1.0], [1.0])
    d1, d2 = P.scaling(qp.Q, qp.A, ruiz_iters=10, pock_chambolle=False)
    assert math.isclose(d2[0], 0.5, rel_tol=1e-15)
    assert math.isclose(d1[0], 2.0 ** (1 - 2.0 ** -9), rel_tol=1e-14)
    a = 2.0 ** (-2.0 ** -9)
    d1, d2 = P.scaling(qp.Q, qp.A, ruiz_iters=10, pock_chambolle=True)
    assert math.isclose(d2[0], 0.5 / math.sqrt(1.0 + a), rel_tol=1e-14)
    assert math.isclose(d1[0], 2.0 ** (1 - 2.0 ** -9) / math.sqrt(a), rel_tol=1e-14)


def test_pock_chambolle_alone_closed_form():
    # Q = I3, A = [[1, 1, 0], [0, 1, -1]]: every entry has magnitude 1, so the
    # 1-norms are the entry counts: variables 2, 3, 2 (Q's diagonal plus A's
    # column), constraints 2, 2.
    qp = _qp(np.eye(3), [[1.0, 1.0, 0.0], [0.0, 1.0, -1.0]], [1.0, 1.0], [0.0, 0.0, 0.0])
    d1, d2 = P.scaling(qp.Q, qp.A, ruiz_iters=0, pock_chambolle=True)
    np.testing.assert_allclose(d2, [1 / math.sqrt(2), 1 / math.sqrt(3), 1 / math.sqrt(2)], rtol=1e-15)
    np.testing.assert_allclose(d1, [1 / math.sqrt(2), 1 / math.sqrt(2)], rtol=1e-15)
    # no step at all leaves the identity
    d1, d2 = P.scaling(qp.Q, qp.A, ruiz_iters=0, pock_chambolle=False)
    assert np.all(d1 == 1.0) and np.all(d2 == 1.0)


def test_ruiz_equilibrates_every_row_and_column_of_the_scaled_blocks():
    # Ruiz equilibration converges to a matrix whose rows and columns all have
    # largest magnitude 1.  Checked on the blocks of the scaled problem (Q~ and
    # A~ from scale_qp, not the K the factors were computed on), so a wrong
    # orientation of A or of a factor fails here.
    qp = I.random_qp(n=300, m=120, r_rows=150, q_density=0.03, a_density=0.05, family=1, instance=3)
    qp.A.val[:] *= np.exp(np.random.default_rng(7).uniform(-4, 4, qp.A.nnz))  # badly scaled rows
    d1, d2 = P.scaling(qp.Q, qp.A, ruiz_iters=60, pock_chambolle=False)
    s = P.scale_qp(qp, d1, d2)
    Qh, Ah = abs(s.Q.to_scipy()), abs(s.A.to_scipy())
    var_max = np.maximum(Qh.max(axis=1).toarray().ravel(), Ah.max(axis=0).toarray().ravel())
    con_max = Ah.max(axis=1).toarray().ravel()
    np.testing.assert_allclose(var_max, 1.0, rtol=1e-9)
    np.testing.assert_allclose(con_max, 1.0, rtol=1e-9)
    # the scaled Q stays exactly symmetric (each entry times d_i d_j)
    Qd = s.Q.to_scipy()
    assert (Qd != Qd.T).nnz == 0


def test_empty_rows_and_columns_keep_factor_one():
    # variable 2 appears nowhere (zero column of Q and A); constraint 1 is an
    # all-zero row
    Q = np.diag([2.0, 3.0, 0.0])
    A = np.array([[1.0, -2.0, 0.0], [0.0, 0.0, 0.0]])
    qp = _qp(Q, A, [1.0, 1.0], [1.0, -1.0, 0.0])
    d1, d2 = P.scaling(qp.Q, qp.A)
    assert d2[2] == 1.0 and d1[1] == 1.0
    assert np.all(np.isfinite(d1)) and np.all(np.isfinite(d2)) and np.all(d1 > 0) and np.all(d2 > 0)


def test_solution_maps_back_to_the_unscaled_optimum():
    # The rescaling is a change of variables: x = D2 x~, y = D1 y~ solves the
    # original problem.  A wrong direction of b~, c~, x or y fails here.
    for qp in (I.tiny_qp(6, 10, instance=4), I.random_qp(n=200, m=80, r_rows=100, q_density=0.05,
                                                         a_density=0.05, family=1, instance=5)):
        ref = O.solve(qp, O.Settings(tol=1e-10, max_iters=400_000))
        x, y, r, d1, d2 = P.solve(qp, O.Settings(tol=1e-10, max_iters=400_000))
        assert ref.status == O.OPTIMAL and r.status == O.OPTIMAL
        assert np.linalg.norm(x - ref.x) <= 1e-6 * max(1.0, np.linalg.norm(ref.x))
        k = O.kkt(qp, x, y)
        assert k["rel_kkt"] <= 1e-7
        assert abs(k["primal_obj"] - ref.primal_obj) <= 1e-8 * (1 + abs(ref.primal_obj))
        # the scaled objective equals the original one at corresponding points
        assert math.isclose(r.primal_obj, ref.primal_obj, rel_tol=1e-7, abs_tol=1e-9)


W = ([[2.0, 0.0], [0.0, 1.0]], [[1.0, 1.0]], [1.0], [-2.0, -1.0])  # the hand-worked example


def test_termination_is_measured_on_the_callers_problem():
    # Example W: at (0, 0) relKKT = r_dual = ||c||/(1 + ||c||) = 2/3.  Scaled
    # by D2 = diag(2, 1), D1 = 4 the copy has c~ = (-4, -1), so its own relKKT
    # at (0, 0) is 4/5; scaled by D2 = diag(1/2, 1/2), D1 = 1 it has
    # c~ = (-1, -1/2) and relKKT 1/2.  With tol between the two values the
    # start point passes or fails on the caller's 2/3 alone.
    qp = _qp(*W)
    x, y, r = P.solve_scaled(qp, np.array([4.0]), np.array([2.0, 1.0]), O.Settings(tol=0.7))
    assert r.status == O.OPTIMAL and r.iters == 0
    assert math.isclose(r.rel_kkt, 2.0 / 3.0, rel_tol=1e-15) and math.isclose(r.r_dual, 2.0 / 3.0, rel_tol=1e-15)
    x, y, r = P.solve_scaled(qp, np.array([1.0]), np.array([0.5, 0.5]), O.Settings(tol=0.6))
    assert r.status == O.OPTIMAL and r.iters > 0 and r.rel_kkt <= 0.6
    # the reported pieces are those of the returned point on the caller's data
    k = O.kkt(qp, x, y)
    assert math.isclose(r.rel_kkt, k["rel_kkt"], rel_tol=1e-12)
    # a start at W's optimum (x*, y*) = ((2/3, 1/3), 2/3) maps to the scaled
    # copy and back unchanged: relKKT 0 there, no iteration
    x, y, r = P.solve_scaled(qp, np.array([4.0]), np.array([2.0, 1.0]), O.Settings(tol=1e-12),
                             x0=[2.0 / 3.0, 1.0 / 3.0], y0=[2.0 / 3.0])
    assert r.iters == 0 and r.rel_kkt <= 1e-15
    np.testing.assert_allclose(x, [2.0 / 3.0, 1.0 / 3.0], rtol=1e-15)
    # to tight tolerance the scaled solve reaches W's exact optimum
    x, y, r = P.solve_scaled(qp, np.array([4.0]), np.array([2.0, 1.0]), O.Settings(tol=1e-12))
    np.testing.assert_allclose(x, [2.0 / 3.0, 1.0 / 3.0], rtol=1e-10)
    np.testing.assert_allclose(y, [2.0 / 3.0], rtol=1e-10)


def test_row_scaled_manufactured_optimum_to_tolerance():
    # A manufactured QP (exact x*, y*) with rows of A and b rescaled by
    # exp(U[-3, 3]): the preconditioned solve must meet the tolerance on the
    # caller's data and land on the exact optimum.
    qp = I.row_scaled(I.manufactured(n=300, m=150, q_density=0.03, a_density=0.03, instance=2))
    x, y, r, d1, d2 = P.solve(qp, O.Settings(tol=1e-9, max_iters=200_000))
    assert r.status == O.OPTIMAL and r.rel_kkt <= 1e-9
    assert np.linalg.norm(x - qp.x_star) <= 1e-6 * np.linalg.norm(qp.x_star)
    assert np.all(y >= 0.0)
    np.testing.assert_allclose(qp.A.to_scipy().T @ y, qp.A.to_scipy().T @ qp.y_star, rtol=0,
                               atol=1e-5 * np.abs(qp.A.to_scipy().T @ qp.y_star).max())


def test_scaled_termination_mistake_is_caught(tmp_path):
    # the former reading (relKKT of the scaled copy) planted in the C oracle
    from test_oracle_mutations import build_mutant
    O.use_library(build_mutant(tmp_path, "    if (!o) {\n        or_kkt(Q, A, b, c, x, y, out);",
                               "    if (1) {\n        or_kkt(Q, A, b, c, x, y, out);"))
    try:
        with pytest.raises(AssertionError):
            test_termination_is_measured_on_the_callers_problem()
    finally:
        O.use_library(None)


# ------------------------------------------------- planted mistakes are caught
# Each case plants one mistake in a copy of oracle/precondition.py, loads the
# copy as a module in place of the real one, and checks that at least one pin
# above fails against it.

_SRC = pathlib.Path(P.__file__).read_text()

MUTATIONS = [
    ("Ruiz step uses the 1-norm", "f = _factor(abs(K).max(axis=1).toarray().ravel())",
     "f = _factor(np.asarray(abs(K).sum(axis=1)).ravel())"),
    ("Pock-Chambolle step uses the maximum", "f = _factor(np.asarray(abs(K).sum(axis=1)).ravel())",
     "f = _factor(abs(K).max(axis=1).toarray().ravel())"),
    ("factor without the square root", "out[pos] = 1.0 / np.sqrt(s[pos])", "out[pos] = 1.0 / s[pos]"),
    ("zero rows get factor 0", "out = np.ones_like(s)", "out = np.zeros_like(s)"),
    ("one-sided rescaling of K", "K.data * (f[K.row] * f[K.col])", "K.data * f[K.row]"),
    ("A~ drops the column factor", "As.data * (d1[As.row] * d2[As.col])", "As.data * d1[As.row]"),
    ("b~ divided by D1", "b=qp.b * d1", "b=qp.b / d1"),
    ("c not scaled", "c=qp.c * d2", "c=qp.c"),
    ("x mapped back the wrong way", "return d2 * r.x, d1 * r.y", "return r.x / d2, d1 * r.y"),
    ("relKKT taken on the scaled copy", "original=(qp, d1, d2))", "original=None)"),
    ("start point mapped the wrong way", "np.asarray(x0, float) / d2", "np.asarray(x0, float) * d2"),
]

PINS = [test_one_by_one_closed_form, test_pock_chambolle_alone_closed_form, test_empty_rows_and_columns_keep_factor_one,
        test_ruiz_equilibrates_every_row_and_column_of_the_scaled_blocks, test_solution_maps_back_to_the_unscaled_optimum,
        test_termination_is_measured_on_the_callers_problem]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(name, old, new, monkeypatch):
    assert _SRC.count(old) == 1, name
    mutant = types.ModuleType("precondition_mutant")
    mutant.__file__ = P.__file__
    exec(compile(_SRC.replace(old, new), "precondition_mutant", "exec"), mutant.__dict__)
    monkeypatch.setitem(globals(), "P", mutant)
    for pin in PINS:
        try:
            pin()
        except Exception:
            return
    pytest.fail(f"no pin caught the planted mistake: {name}")
