"""Accuracy of the FP64 and the FP32-product modes against the FP64 oracle
(run to relKKT 1e-9, or the exact optimum of a manufactured instance), each
family solved to relKKT 1e-6 in both modes.  Needs a GPU; prints one JSON
object.  Run from the repository root:  python tests/precision_report.py

A report, not a test (pytest does not collect it): the oracle may be used here
and not in the benchmark."""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import oracle as O  # noqa: E402
from paper_2405_16160_amd import instances as I, pdhcg  # noqa: E402


def main():
    cases = [("tiny random n=1000", I.random_qp(family=1, instance=0), None),
             ("random n=1e5 (benchmark instance)", I.random_qp(100_000, 50_000, 50_000, 2e-5, 2e-4, family=2), None),
             ("manufactured n=1e5 (exact optimum)", I.manufactured(100_000, 50_000, 2e-5, 2e-4, r_rows=50_000,
                                                                   family=41), "exact"),
             ("MPC n=1500 m=5000", I.mpc_qp(0), None),
             ("portfolio n=355 (dense Q)", I.portfolio_qp(0, nmax=400), None)]
    out = {}
    for name, qp, kind in cases:
        print(f"[precision] {name}", file=sys.stderr, flush=True)
        if kind == "exact":
            xr, fr = qp.x_star, 0.5 * qp.x_star @ (qp.Q.to_scipy() @ qp.x_star) + qp.c @ qp.x_star
        else:
            ref = O.solve(qp, O.Settings(tol=1e-9, max_iters=1_000_000))
            xr, fr = ref.x, ref.primal_obj
        row = {}
        for prec in (0, 1):
            sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=1e-6, precision=prec, max_iters=1_000_000))
            x, y, r = sol.solve()
            sol.close()
            x = x.cpu().numpy()
            k = O.kkt(qp, x, y.cpu().numpy())
            row["fp64" if prec == 0 else "fp32_products"] = {
                "rel_kkt_fp64_data": k["rel_kkt"], "x_rel_err": float(np.linalg.norm(x - xr) / np.linalg.norm(xr)),
                "obj_rel_err": abs(k["primal_obj"] - fr) / (1 + abs(fr)), "iters": r["iters"]}
        out[name] = row
    print(json.dumps({"report": "precision modes vs the FP64 oracle at relKKT 1e-6", "cases": out}))


if __name__ == "__main__":
    main()
