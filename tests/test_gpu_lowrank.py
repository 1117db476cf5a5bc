"""GPU parity of the single-QP path with Q in low-rank form, Q = P P' + diag(d)
(Sec. 2, low-rank acceleration of Q: every product with Q formed as
P (P' v) + d v), through the C ABI (pdhcg_create_lowrank), against the FP64
oracle run on the explicit Q = P P' + diag(d):

  * the worked example W written as P = [1; 0], d = (1, 1) (Q = diag(2, 1)):
    the first iteration's closed form;
  * random sparse P (n = 2000, k = 300) in both precisions: the full parity
    contract at relKKT 1e-6, and iteration and CG-step counts equal (within
    2 % or 64) to those of the same solve with Q given explicitly;
  * d = 0 with P of full row rank (n = 60, k = 90);
  * the n = 1e5 set of the low-rank benchmark mode to 1e-4 (relKKT
    recomputed by the oracle on the explicit Q);
  * the settings the low-rank form does not take are rejected."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import oracle as O
from paper_2405_16160_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_16160_amd import pdhcg  # noqa: E402


def say(msg):
    print(msg, flush=True)


def solve(qp, lowrank=None, **kw):
    sol = pdhcg.Solver(qp, pdhcg.Settings(**kw), lowrank=lowrank)
    x, y, r = sol.solve()
    sol.close()
    return x.cpu().numpy(), y.cpu().numpy(), r


def contract(qp, x, y, ref, tol):
    k = O.kkt(qp, x, y)
    assert k["rel_kkt"] <= tol * (1 + 1e-6), k
    assert np.all(y >= 0)
    assert abs(k["primal_obj"] - ref.primal_obj) / (1 + abs(ref.primal_obj)) <= 1e-6
    assert np.linalg.norm(x - ref.x) / max(np.linalg.norm(ref.x), 1e-300) <= 1e-4
    return k


def test_worked_example_first_iteration():
    say("[lowrank] W as P = [1; 0], d = (1, 1)")
    qp = I.QP(I.CSR.from_scipy(sp.csr_matrix(np.diag([2.0, 1.0]))), I.CSR.from_scipy(sp.csr_matrix([[1.0, 1.0]])),
              np.array([1.0]), np.array([-2.0, -1.0]))
    P = I.CSR.from_scipy(sp.csr_matrix(np.array([[1.0], [0.0]])))
    x, y, r = solve(qp, lowrank=(P, np.array([1.0, 1.0])), tol_rel_kkt=1e-14, max_iters=1, max_cg_iters=2,
                    cg_eps_factor=0.0, eval_period=1000)
    s2 = math.sqrt(2.0)
    assert np.allclose(x, [s2 - 1, 1 / (1 + 2 * s2)], atol=1e-14)
    assert y[0] == pytest.approx((2 * x.sum() - 1) / (2 * s2), abs=1e-14)
    x, y, r = solve(qp, lowrank=(P, np.array([1.0, 1.0])), tol_rel_kkt=1e-10)
    assert r["status"] == 0 and np.allclose(x, [2 / 3, 1 / 3], atol=1e-8)


@pytest.mark.parametrize("precision", [0, 1])
def test_random_lowrank_parity(precision):
    say(f"[lowrank] n=2000 k=300 precision={precision}")
    qp, P, d = I.lowrank_qp(n=2000, m=1000, k=300, p_density=0.01, a_density=0.005, instance=1)
    ref = O.solve(qp, O.Settings(tol=1e-9, max_iters=400_000))
    assert ref.status == O.OPTIMAL
    x, y, r = solve(qp, lowrank=(P, d), tol_rel_kkt=1e-6, precision=precision)
    xe, ye, re_ = solve(qp, tol_rel_kkt=1e-6, precision=precision, cg_form=2)
    say(f"  low-rank iters={r['iters']} cg={r['cg_iters_total']}; explicit Q iters={re_['iters']} "
        f"cg={re_['cg_iters_total']}; nnz(P)={P.nnz} nnz(Q)={qp.Q.nnz}")
    assert r["status"] == 0
    k = contract(qp, x, y, ref, 1e-6)
    assert r["rel_kkt"] == pytest.approx(k["rel_kkt"], rel=1e-6, abs=1e-12)
    assert abs(r["iters"] - re_["iters"]) <= max(64, 0.02 * re_["iters"])
    assert abs(r["cg_iters_total"] - re_["cg_iters_total"]) <= max(64, 0.02 * re_["cg_iters_total"])


def test_lowrank_at_256_thread_workgroups():
    """The low-rank products in the cooperative kernels compiled for
    256-thread workgroups (forced; the planner keeps 512 for a low-rank Q)."""
    say("[lowrank] n=2000 k=300 threads=256")
    qp, P, d = I.lowrank_qp(n=2000, m=1000, k=300, p_density=0.01, a_density=0.005, instance=1)
    ref = O.solve(qp, O.Settings(tol=1e-9, max_iters=400_000))
    x, y, r = solve(qp, lowrank=(P, d), tol_rel_kkt=1e-6, precision=1, threads=256)
    say(f"  iters={r['iters']} cg={r['cg_iters_total']}")
    assert r["status"] == 0
    contract(qp, x, y, ref, 1e-6)


def test_zero_diagonal_full_row_rank():
    say("[lowrank] d = 0, n=60 k=90")
    qp, P, d = I.lowrank_qp(n=60, m=30, k=90, p_density=0.2, a_density=0.2, instance=2)
    Pd = P.to_scipy().toarray()
    Qd = Pd @ Pd.T
    qp0 = I.QP(I.CSR.from_scipy(sp.csr_matrix((Qd + Qd.T) * 0.5)), qp.A, qp.b, qp.c)   # exactly symmetric
    ref = O.solve(qp0, O.Settings(tol=1e-10, max_iters=400_000))
    assert ref.status == O.OPTIMAL
    x, y, r = solve(qp0, lowrank=(P, None), tol_rel_kkt=1e-8)
    assert r["status"] == 0
    assert O.kkt(qp0, x, y)["rel_kkt"] <= 1e-8 * (1 + 1e-6)
    assert np.linalg.norm(x - ref.x) <= 1e-5 * max(1.0, np.linalg.norm(ref.x))


def test_benchmark_set_to_1e4():
    say("[lowrank] n=1e5 k=2000, tol 1e-4, FP32 products")
    qp, P, d = I.lowrank_qp(n=100_000, m=50_000, k=2_000, instance=0)
    x, y, r = solve(qp, lowrank=(P, d), tol_rel_kkt=1e-4, precision=1)
    k = O.kkt(qp, x, y)
    say(f"  status={r['status_name']} iters={r['iters']} cg={r['cg_iters_total']} kernel={r['kernel_s']:.3f}s "
        f"relKKT={k['rel_kkt']:.2e} nnz(P)={P.nnz} nnz(Q)={qp.Q.nnz}")
    assert r["status"] == 0
    assert k["rel_kkt"] <= 1e-4 * (1 + 1e-6)
    assert r["rel_kkt"] == pytest.approx(k["rel_kkt"], rel=1e-6, abs=1e-12)


def test_rejected_settings():
    qp, P, d = I.lowrank_qp(n=200, m=100, k=40, p_density=0.05, a_density=0.02, instance=3)
    for bad in (dict(ruiz_iters=10), dict(pock_chambolle=1), dict(step_rule=1)):
        with pytest.raises(pdhcg.PdhcgError) as e:
            pdhcg.Solver(qp, pdhcg.Settings(**bad), lowrank=(P, d))
        assert e.value.code == -1
    with pytest.raises(pdhcg.PdhcgError):
        pdhcg.Solver(qp, pdhcg.Settings(), lowrank=(P, -d))
    sol = pdhcg.Solver(qp, pdhcg.Settings(), lowrank=(P, d))
    with pytest.raises(pdhcg.PdhcgError):
        sol.spmv(0, np.ones(qp.n))
    with pytest.raises(pdhcg.PdhcgError):
        sol.set_settings(pdhcg.Settings(step_rule=1))
    sol.close()
