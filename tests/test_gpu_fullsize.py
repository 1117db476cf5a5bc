"""Whole solves at the power-law set's full size (n = 2e6, m = 1e6, A rows with
a Pareto(1.5) length law of mean 8 clipped to [1, 5000]; the scale of the
paper's large synthetic experiments, Sec. 5.1), through the C ABI, in the
launch configuration the benchmark uses (FP32 products, diagonal
preconditioning, relKKT on the caller's problem):

  * the manufactured instance with the same Q and A law and a known optimum
    (x*, y*) is solved to relKKT 1e-6 in both precision modes: x within 1e-4
    of x* and the objective within 1e-6 (the precision error of each mode is
    printed and bounded);
  * the generated instance is solved to relKKT 1e-4, and the oracle's FP64
    relKKT of the returned point (recomputed on the CPU) is <= 1e-4.

The oracle's whole solve is too slow at this size; the manufactured optimum
and the FP64 recomputation of relKKT stand in for it.

The benchmark batch (4 096 preconditioned portfolio QPs, factored Q, FP32
products, tol 1e-4, the autotuner's workgroup size) is held to the same kind
of checks: every instance OPTIMAL, relKKT recomputed by the oracle on a
sample of 256 instances, the objective against the oracle's optimum on eight
of them."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_16160_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_16160_amd import pdhcg  # noqa: E402

PRE = dict(ruiz_iters=10, pock_chambolle=1)


def say(msg):
    print(msg, flush=True)


def solve(qp, **kw):
    sol = pdhcg.Solver(qp, pdhcg.Settings(**kw))
    x, y, r = sol.solve()
    sol.close()
    return x.cpu().numpy(), y.cpu().numpy(), r


@pytest.fixture(scope="module")
def manufactured():
    say("[fullsize] generating the manufactured power-law QP n=2e6 m=1e6")
    return I.powerlaw_manufactured()


@pytest.mark.parametrize("precision", [1, 0])
def test_powerlaw_manufactured_full_size(manufactured, precision):
    qp = manufactured
    xs = qp.x_star
    fs = 0.5 * xs @ (qp.Q.to_scipy() @ xs) + qp.c @ xs
    say(f"[fullsize] manufactured n=2e6 precision={precision} tol 1e-6")
    x, y, r = solve(qp, tol_rel_kkt=1e-6, precision=precision, max_iters=200_000, **PRE)
    k = O.kkt(qp, x, y)
    xerr = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    ferr = abs(k["primal_obj"] - fs) / (1 + abs(fs))
    say(f"  status={r['status_name']} iters={r['iters']} cg={r['cg_iters_total']} kernel={r['kernel_s']:.2f}s "
        f"relKKT(oracle)={k['rel_kkt']:.2e} |x-x*|/|x*|={xerr:.2e} objective error={ferr:.2e}")
    assert r["status"] == 0
    assert k["rel_kkt"] <= 1e-6 * (1 + 1e-6)
    assert r["rel_kkt"] == pytest.approx(k["rel_kkt"], rel=1e-6, abs=1e-12)
    assert np.all(y >= 0)
    assert xerr <= 1e-4
    assert ferr <= 1e-6


def test_powerlaw_generated_full_size_to_1e4():
    say("[fullsize] generated power-law QP n=2e6 m=1e6, tol 1e-4, both precisions")
    qp = I.powerlaw_qp()
    xs = {}
    for precision in (1, 0):
        x, y, r = solve(qp, tol_rel_kkt=1e-4, precision=precision, **PRE)
        k = O.kkt(qp, x, y)
        say(f"  precision={precision} status={r['status_name']} iters={r['iters']} kernel={r['kernel_s']:.3f}s "
            f"relKKT reported={r['rel_kkt']:.3e} oracle={k['rel_kkt']:.3e}")
        assert r["status"] == 0
        assert k["rel_kkt"] <= 1e-4 * (1 + 1e-6)
        assert r["rel_kkt"] == pytest.approx(k["rel_kkt"], rel=1e-6, abs=1e-12)
        assert np.all(y >= 0)
        xs[precision] = x
    d = np.linalg.norm(xs[1] - xs[0]) / np.linalg.norm(xs[0])
    say(f"  |x_fp32 - x_fp64| / |x_fp64| = {d:.2e}")


def test_portfolio_batch_in_the_benchmark_configuration():
    """The benchmark batch itself, in the launch configuration bench.py times:
    the 4 096 portfolio QPs with Q in factored form, per-instance Ruiz +
    Pock-Chambolle preconditioning, FP32 products, relKKT <= 1e-4 on each
    caller's problem, the workgroup size the batch autotuner picks.  Every
    instance ends OPTIMAL with y >= 0.  On every 16th instance (256 of them,
    all sizes) the oracle recomputes relKKT from the dense Q of the same QP:
    <= 1e-4 and equal to the reported value.  On the first eight of those with
    n <= 400 the oracle's own preprocessed FP64 solve run to 1e-9 gives the
    optimum, and the objective is within 2e-4 (1 + |f*|), what the gap term of
    relKKT <= 1e-4 allows (the oracle stopped at 1e-4 is itself up to 3.4e-5
    off on this family)."""
    from oracle import precondition as PC
    say("[fullsize] 4096 portfolio QPs, factored, preconditioned, FP32 products, tol 1e-4")
    pairs = [I.portfolio_lowrank(i) for i in range(4096)]
    s = pdhcg.Settings(tol_rel_kkt=1e-4, precision=1, max_iters=200_000, **PRE)
    b = pdhcg.Batch([q for q, _ in pairs], s, lowrank=[f for _, f in pairs])
    t = b.autotune(reps=1)
    x, y, rs = b.solve()
    xs, ys = b.split(x, y)
    b.close()
    say(f"  autotuner {t}; kernel {rs[0]['kernel_s']:.3f} s; iterations mean "
        f"{np.mean([r['iters'] for r in rs]):.1f} max {max(r['iters'] for r in rs)}")
    assert all(r["status"] == 0 for r in rs)
    assert all(np.all(yi >= 0) for yi in ys)
    refs = 0
    for i in range(0, 4096, 16):
        qp = I.portfolio_qp(i)   # the same QP with Q = F F' + diag(d) formed densely
        k = O.kkt(qp, xs[i], ys[i])
        assert k["rel_kkt"] <= 1e-4 * (1 + 1e-6), (i, k)
        assert rs[i]["rel_kkt"] == pytest.approx(k["rel_kkt"], rel=1e-6, abs=1e-12)
        if qp.n <= 400 and refs < 8:
            _, _, rr, _, _ = PC.solve(qp, O.Settings(tol=1e-9, max_iters=1_000_000))
            assert rr.status == O.OPTIMAL
            err = abs(k["primal_obj"] - rr.primal_obj) / (1 + abs(rr.primal_obj))
            say(f"  instance {i} n={qp.n}: objective error {err:.2e}")
            assert err <= 2e-4
            refs += 1
    assert refs == 8
