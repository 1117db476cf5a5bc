"""Learned warm start end to end on the MPC family (small scale): PDHCG
solutions from the batched solver train the bfloat16 network on the GPU; on
held-out family members the warm-started solves meet the same relKKT test
(checked by the FP64 oracle) in fewer iterations than cold starts."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_16160_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_16160_amd import pdhcg, warmstart as W  # noqa: E402


def say(msg):
    print(msg, flush=True)


def test_learned_warm_start_gains_over_cold_start():
    fam = I.mpc_family()
    plus, minus = W.pair_index(fam)
    s = pdhcg.Settings(tol_rel_kkt=1e-4)
    say("[warmstart] 3000 training solves")
    th, X, Y, rs, secs = W.solve_family(fam, range(3000), pdhcg.Settings(tol_rel_kkt=1e-6))
    assert all(r["status"] == 0 for r in rs)
    Y = W.canonical_duals(Y, plus, minus)
    say(f"  solved in {secs:.2f}s; training")
    ws, losses = W.train(th, X, Y, W.DualCode(fam.A.nrows, plus, minus), epochs=40, batch=256, lr=2e-3, log=say)
    assert losses[-1] < 0.5 * losses[0]
    test_ids = range(100_000, 100_200)
    th_t, qps = W.family_qps(fam, test_ids)
    x0, y0 = ws.predict(th_t)
    _, Xc, Yc, rc, tc = W.solve_family(fam, test_ids, s)
    _, Xw, Yw, rw, tw = W.solve_family(fam, test_ids, s, x0s=x0, y0s=y0)
    it_c = np.array([r["iters"] for r in rc])
    it_w = np.array([r["iters"] for r in rw])
    fb = np.mean([r["cold_fallback"] for r in rw])
    say(f"  cold: mean iters {it_c.mean():.1f} ({tc:.3f}s); warm: {it_w.mean():.1f} ({tw:.3f}s); fallback rate {fb:.3f}")
    assert all(r["status"] == 0 for r in rc + rw)
    for i in range(0, 200, 40):   # the same relKKT test, recomputed in FP64 by the oracle
        assert O.kkt(qps[i], Xw[i], Yw[i])["rel_kkt"] <= 1e-4 * (1 + 1e-6)
    assert it_w.mean() < 0.8 * it_c.mean()
