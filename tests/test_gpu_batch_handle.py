"""GPU tests of the reusable batch (pdhcg_batch_create / pdhcg_batch_solve):
repeated solves on device-resident data, device-resident inputs and outputs,
and per-instance diagonal preconditioning (Sec. 4, "Preprocessing") in one
launch for dense and factored Q (Q = F F' + diag(d), the low-rank form of
Sec. 2), each against the FP64 oracle with the full parity contract on the
caller's problem: relKKT recomputed by the oracle <= tol, x within 1e-4 of
the oracle's optimum (run to 1e-9), objective within 1e-6, y >= 0.  On the
portfolio family relKKT <= 1e-6 alone does not always imply the objective bar
(the oracle stopped at 1e-6 is itself up to 1.5e-6 off), so those solves run
to 1e-7."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import precondition as P
from paper_2405_16160_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_16160_amd import pdhcg  # noqa: E402

PRE = dict(ruiz_iters=10, pock_chambolle=1)


def say(msg):
    print(msg, flush=True)


def check_contract(qp, x, y, r, xr, objr, tol):
    assert r["status"] == 0, r
    assert np.all(y >= 0.0)
    k = O.kkt(qp, x, y)
    assert k["rel_kkt"] <= tol * (1 + 1e-6), k
    assert r["rel_kkt"] == pytest.approx(k["rel_kkt"], rel=1e-6, abs=1e-12)
    assert np.linalg.norm(x - xr) / max(np.linalg.norm(xr), 1e-12) <= 1e-4
    assert abs(k["primal_obj"] - objr) / (1 + abs(objr)) <= 1e-6


def test_batch_handle_repeats_and_matches_one_call():
    """Two solves of one packed batch are bit-identical; they equal the
    one-call entry point's; a warm start from the packed device outputs ends
    within one iteration."""
    say("[batch handle] 4 portfolio + 2 random QPs, repeated solves")
    qps = [I.portfolio_qp(i, nmax=300) for i in range(4)] + [I.random_qp(family=1, instance=i) for i in range(2)]
    s = pdhcg.Settings(tol_rel_kkt=1e-6)
    b = pdhcg.Batch(qps, s)
    x1, y1, r1 = b.solve()
    x1, y1 = x1.clone(), y1.clone()
    x2, y2, r2 = b.solve()
    assert torch.equal(x1, x2) and torch.equal(y1, y2)
    assert [r["iters"] for r in r1] == [r["iters"] for r in r2]
    one = pdhcg.solve_batch(qps, s)
    xs, ys = b.split(x1, y1)
    for i, (x, y, r) in enumerate(one):
        assert np.array_equal(xs[i], x) and np.array_equal(ys[i], y)
        assert r["iters"] == r1[i]["iters"]
        assert O.kkt(qps[i], x, y)["rel_kkt"] <= 1e-6 * (1 + 1e-6)
    _, _, r3 = b.solve(x0=x1, y0=y1)
    for a, c in zip(r3, r1):
        assert a["status"] == 0 and a["cold_fallback"] == 0 and a["iters"] <= 1 < c["iters"]
    b.close()


@pytest.mark.parametrize("lowrank", [False, True])
def test_batch_device_inputs_equal_host_inputs(lowrank):
    """CSR, factor and vector inputs handed over as device pointers give the
    same packed data, so the same solve bit for bit."""
    say(f"[batch handle] device-resident inputs, lowrank={lowrank}")
    qps = [I.portfolio_qp(i, nmax=250) for i in range(5)]
    fac = [I.portfolio_factor(i, nmax=250) for i in range(5)] if lowrank else None
    s = pdhcg.Settings(tol_rel_kkt=1e-6, precision=1)
    bh = pdhcg.Batch(qps, s, lowrank=fac)
    bd = pdhcg.Batch(qps, s, lowrank=fac, device_inputs=True)
    xh, yh, rh = bh.solve()
    xd, yd, rd = bd.solve()
    assert torch.equal(xh, xd) and torch.equal(yh, yd)
    assert [r["iters"] for r in rh] == [r["iters"] for r in rd]
    assert all(r["status"] == 0 for r in rd)
    bh.close()
    bd.close()


_REF = {}


def oracle_ref(i, qp):
    if i not in _REF:
        xr, yr, rr, e1, e2 = P.solve(qp, O.Settings(tol=1e-9, max_iters=400_000))
        assert rr.status == O.OPTIMAL
        _REF[i] = (xr, rr.primal_obj, e1, e2)
    return _REF[i]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("form", ["dense", "factored"])
def test_batch_preconditioned_portfolio_vs_oracle(form, precision):
    """Portfolio QPs (n up to 400) preconditioned per instance in one launch:
    D1, D2 equal the oracle's (computed on the dense Q) to rtol 1e-13 in both
    forms, and every solve meets the contract on the caller's problem."""
    say(f"[batch precondition] 6 portfolio QPs, {form} Q, precision={precision}")
    ids = list(range(6))
    qps = [I.portfolio_qp(i, nmax=400) for i in ids]
    fac = [I.portfolio_factor(i, nmax=400) for i in ids] if form == "factored" else None
    b = pdhcg.Batch(qps, pdhcg.Settings(tol_rel_kkt=1e-7, precision=precision, max_iters=400_000, **PRE),
                    lowrank=fac)
    d1, d2 = b.scaling()
    d2s, d1s = b.split(d2, d1)   # per instance: D2 (n), D1 (m)
    x, y, rs = b.solve()
    xs, ys = b.split(x, y)
    for j, qp in enumerate(qps):
        xr, objr, e1, e2 = oracle_ref(ids[j], qp)
        np.testing.assert_allclose(d2s[j], e2, rtol=1e-13, atol=0)
        np.testing.assert_allclose(d1s[j], e1, rtol=1e-13, atol=0)
        say(f"  n={qp.n} status={rs[j]['status_name']} iters={rs[j]['iters']} kkt={rs[j]['rel_kkt']:.2e}")
        check_contract(qp, xs[j], ys[j], rs[j], xr, objr, 1e-7)
    b.close()


@pytest.mark.parametrize("form", ["dense", "factored"])
def test_batch_preconditioned_portfolio_maximum_size(form):
    """The largest size of the portfolio configuration (n = 2000, k = 200)
    beside small instances, preconditioned, FP32 products: the n = 2000 solve
    meets the full contract against the oracle (preconditioned, 1e-9)."""
    say(f"[batch precondition max] n = 2000 + 3 small, {form} Q")
    qps = [I.portfolio_qp(900, n=2000)] + [I.portfolio_qp(i, nmax=120) for i in range(3)]
    fac = ([I.portfolio_factor(900, n=2000)] + [I.portfolio_factor(i, nmax=120) for i in range(3)]
           if form == "factored" else None)
    b = pdhcg.Batch(qps, pdhcg.Settings(tol_rel_kkt=1e-7, precision=1, max_iters=200_000, **PRE), lowrank=fac)
    x, y, rs = b.solve()
    xs, ys = b.split(x, y)
    xr, objr, _, _ = oracle_ref(("max", 900), qps[0])
    say(f"  n=2000 status={rs[0]['status_name']} iters={rs[0]['iters']} kkt={rs[0]['rel_kkt']:.2e}")
    check_contract(qps[0], xs[0], ys[0], rs[0], xr, objr, 1e-7)
    for j in range(1, 4):
        assert rs[j]["status"] == 0
        assert O.kkt(qps[j], xs[j], ys[j])["rel_kkt"] <= 1e-7 * (1 + 1e-6)
    b.close()
