"""Learned warm start end to end on the MPC family (small scale): PDHCG
solutions from the batched solver train the bfloat16 network on the GPU; on
held-out family members the warm-started solves meet the same relKKT test
(checked by the FP64 oracle) in fewer iterations than cold starts."""
import dataclasses

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
    say("[warmstart] 8000 training solves")
    th, X, Y, rs, secs = W.solve_family(fam, range(8000), pdhcg.Settings(tol_rel_kkt=1e-6))
    assert all(r["status"] == 0 for r in rs)
    Y = W.canonical_duals(Y, plus, minus)
    say(f"  solved in {secs:.2f}s; training")
    ws, losses = W.train(th, X, Y, W.DualCode(fam.A.nrows, plus, minus), epochs=400, batch=256, lr=1e-3)
    say(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 0.1 * losses[0]
    s = pdhcg.Settings(tol_rel_kkt=1e-4)
    v = W.validate(fam, ws, range(100_000, 100_200), s)
    say(f"  cold: mean iters {v['cold_iters']:.1f} ({v['cold_s']:.3f}s); warm: {v['warm_iters']:.1f} ({v['warm_s']:.3f}s)")
    assert v["solved"] == v["count"]
    assert v["pays"]
    assert v["warm_iters"] < 0.9 * v["cold_iters"]
    # the warm-started points meet the same relKKT test, recomputed in FP64 by the oracle
    ids = range(100_000, 100_200, 40)
    th_t, qps = W.family_qps(fam, ids)
    x0, y0 = ws.predict(th_t)
    _, Xw, Yw, rw, _ = W.solve_family(fam, ids, dataclasses.replace(s, warm_fallback=0), x0s=x0, y0s=y0)
    for q, x, y, r in zip(qps, Xw, Yw, rw):
        assert r["status"] == 0 and r["cold_fallback"] == 0
        assert O.kkt(q, x, y)["rel_kkt"] <= 1e-4 * (1 + 1e-6)
    # with the per-instance fallback on, the solves stay correct whichever start they keep
    _, Xf, Yf, rf, _ = W.solve_family(fam, ids, s, x0s=x0, y0s=y0)
    for q, x, y, r in zip(qps, Xf, Yf, rf):
        assert r["status"] == 0
        assert O.kkt(q, x, y)["rel_kkt"] <= 1e-4 * (1 + 1e-6)
