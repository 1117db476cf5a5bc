"""GPU test of pdhcg_solve_batch_noalloc, the allocation-free variant of
pdhcg_solve_batch (every device buffer carved from the library's static
scratch), through the C ABI: on two calls in a row, the second with a smaller
input, and on a preconditioned batch, its iterates, counts and results equal
those of pdhcg_solve_batch on the same inputs, and every returned point meets
relKKT <= tol recomputed by the oracle; a batch larger than the scratch is
rejected on the host with INVALID_ARGUMENT."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2405_16160_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_16160_amd import pdhcg  # noqa: E402


def say(msg):
    print(msg, flush=True)


def compare(qps, settings, tol):
    ref = pdhcg.solve_batch(qps, settings)
    got = pdhcg.solve_batch(qps, settings, noalloc=True)
    for qp, (xr, yr, rr), (x, y, r) in zip(qps, ref, got):
        assert r["status"] == 0 and rr["status"] == 0, (r, rr)
        assert (r["iters"], r["cg_iters_total"], r["restarts"]) == (rr["iters"], rr["cg_iters_total"], rr["restarts"])
        assert np.linalg.norm(x - xr) <= 1e-12 * (1 + np.linalg.norm(xr))
        assert np.linalg.norm(y - yr) <= 1e-12 * (1 + np.linalg.norm(yr))
        assert r["rel_kkt"] == pytest.approx(rr["rel_kkt"], rel=1e-9, abs=1e-15)
        k = O.kkt(qp, x, y)
        assert k["rel_kkt"] <= tol * (1 + 1e-6)
        assert np.all(y >= 0)


def test_noalloc_matches_the_allocating_entry_point():
    s = pdhcg.Settings(tol_rel_kkt=1e-6, precision=1)
    big = [I.portfolio_qp(i, n=n) for i, n in enumerate((300, 120, 57, 200, 90, 64))] + \
          [I.random_qp(n=400, m=200, r_rows=200, q_density=0.02, a_density=0.02, family=1, instance=i) for i in range(3)]
    say(f"[noalloc] call 1: {len(big)} instances, sum n = {sum(q.n for q in big)}")
    compare(big, s, 1e-6)
    small = [I.portfolio_qp(10 + i, n=n) for i, n in enumerate((80, 50))] + \
            [I.random_qp(n=150, m=60, r_rows=60, q_density=0.05, a_density=0.05, family=1, instance=9)]
    say(f"[noalloc] call 2 (smaller): {len(small)} instances, sum n = {sum(q.n for q in small)}")
    compare(small, s, 1e-6)
    say("[noalloc] call 3: preconditioned, FP64")
    pre = pdhcg.Settings(tol_rel_kkt=1e-6, precision=0, ruiz_iters=10, pock_chambolle=1)
    compare(small + big[:2], pre, 1e-6)


def test_noalloc_rejects_a_batch_beyond_the_scratch():
    qp = I.portfolio_qp(0, n=2000)   # dense Q: 32 MB of FP64 values, 16 MB of FP32 copies, plus A and vectors
    say("[noalloc] oversized batch is rejected on the host")
    with pytest.raises(pdhcg.PdhcgError) as e:
        pdhcg.solve_batch([qp, qp], pdhcg.Settings(precision=1, ruiz_iters=10, pock_chambolle=1), noalloc=True)
    assert e.value.code == -1 and "static scratch" in str(e.value)
