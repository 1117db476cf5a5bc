"""Accuracy of the two precision modes (FP64 throughout, and FP32 matrix values
and gathered vectors with FP64 accumulation, scalars and termination test)
against the FP64 oracle, through the C ABI: each family solved in both modes,
each result held to the parity contract (relKKT recomputed by the oracle
against the FP64 data <= tol, x within 1e-4 of the oracle's optimum run to
1e-9 (or of the exact optimum of a manufactured instance), objective within
1e-6, y >= 0), the error of each mode printed.  The MPC and portfolio
families run to 1e-7: on them relKKT <= 1e-6 alone does not imply the
objective bar (the oracle stopped at 1e-6 is itself up to 1.5e-6 off)."""
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


CASES = {
    "tiny random n=1000": (lambda: I.random_qp(family=1, instance=0), 1e-6),
    "random n=1e5": (lambda: I.random_qp(100_000, 50_000, 50_000, 2e-5, 2e-4, family=2), 1e-6),
    "manufactured n=1e5": (lambda: I.manufactured(100_000, 50_000, 2e-5, 2e-4, r_rows=50_000, family=41), 1e-6),
    "MPC n=1500 m=5000": (lambda: I.mpc_qp(0), 1e-7),
    "portfolio n=355": (lambda: I.portfolio_qp(0, nmax=400), 1e-7),
}


@pytest.mark.parametrize("name", list(CASES))
def test_precision_modes_against_the_oracle(name):
    make, tol = CASES[name]
    qp = make()
    if qp.x_star is not None:
        xr = qp.x_star
        fr = 0.5 * xr @ (qp.Q.to_scipy() @ xr) + qp.c @ xr
    else:
        ref = O.solve(qp, O.Settings(tol=1e-9, max_iters=1_000_000))
        assert ref.status == O.OPTIMAL
        xr, fr = ref.x, ref.primal_obj
    for precision in (0, 1):
        sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=tol, precision=precision, max_iters=1_000_000))
        x, y, r = sol.solve()
        sol.close()
        x, y = x.cpu().numpy(), y.cpu().numpy()
        k = O.kkt(qp, x, y)
        xerr = np.linalg.norm(x - xr) / np.linalg.norm(xr)
        ferr = abs(k["primal_obj"] - fr) / (1 + abs(fr))
        say(f"[precision] {name} mode={'fp64' if precision == 0 else 'fp32-products'} iters={r['iters']} "
            f"relKKT={k['rel_kkt']:.2e} x err={xerr:.2e} objective err={ferr:.2e}")
        assert r["status"] == 0
        assert k["rel_kkt"] <= tol * (1 + 1e-6)
        assert np.all(y >= 0)
        assert xerr <= 1e-4
        assert ferr <= 1e-6
