"""GPU parity of the HIP library (through its C ABI) against the FP64 CPU oracle.

Contract (strictly convex instances): the GPU point's relKKT, recomputed by the
oracle against the FP64 data, is <= tol; relative objective difference to the
oracle run at relKKT <= 1e-9 is <= 1e-6; ||x - x_or|| / ||x_or|| <= 1e-4.  The
dual y is not unique (+/- row pairs, degenerate rows), so only what is unique
at the optimum is compared: A'y = -(Qx* + c) and b'y; y >= 0 is checked.
"""
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


_REF = {}


def oracle_ref(qp, key):
    if key not in _REF:
        _REF[key] = O.solve(qp, O.Settings(tol=1e-9, max_iters=400_000))
        assert _REF[key].status == O.OPTIMAL
    return _REF[key]


def check_contract(qp, x, y, ref, tol=1e-6, xtol=1e-4, objtol=1e-6):
    x = np.asarray(x)
    y = np.asarray(y)
    k = O.kkt(qp, x, y)
    assert k["rel_kkt"] <= tol * (1 + 1e-6), k
    assert np.all(y >= 0.0)
    assert abs(k["primal_obj"] - ref.primal_obj) / (1 + abs(ref.primal_obj)) <= objtol
    assert np.linalg.norm(x - ref.x) / max(np.linalg.norm(ref.x), 1e-300) <= xtol
    if qp.m:
        aty, aty_r = O.matvec_t(qp.A, y), O.matvec_t(qp.A, ref.y)
        assert np.linalg.norm(aty - aty_r) / (1 + np.linalg.norm(aty_r)) <= 1e-3
    return k


def gpu_solve(qp, **kw):
    s = pdhcg.Settings(**kw)
    sol = pdhcg.Solver(qp, s)
    x, y, r = sol.solve()
    info = sol.plan_info()
    sol.close()
    return x.cpu().numpy(), y.cpu().numpy(), r, info


# ------------------------------------------------------------- SpMV kernels

@pytest.mark.parametrize("case", ["tiny", "powerlaw", "large"])
def test_spmv_parity(case):
    say(f"[spmv] case={case}")
    if case == "tiny":
        qp = I.random_qp(family=1, instance=0)
    elif case == "powerlaw":
        qp = I.powerlaw_qp(60_000, 30_000, family=3, instance=1)   # rows up to 5000 nnz: long-row path
    else:
        qp = I.random_qp(100_000, 50_000, 50_000, 2e-5, 2e-4, family=2)
    sol = pdhcg.Solver(qp)
    rng = np.random.default_rng(7)
    xn, xm = rng.standard_normal(qp.n), rng.standard_normal(qp.m)
    for which, M, v in ((0, qp.Q, xn), (1, qp.A, xn), (2, I.CSR.from_scipy(qp.A.to_scipy().T), xm)):
        ref = O.matvec(M, v)
        got = sol.spmv(which, v).cpu().numpy()
        scale = O.matvec(I.CSR(M.nrows, M.ncols, M.rowptr, M.col, np.abs(M.val)), np.abs(v)) + 1e-300
        err = np.max(np.abs(got - ref) / scale)
        say(f"  which={which} fp64 max rel err={err:.2e}")
        assert err <= 1e-14
        got32 = sol.spmv(which, v, precision=1).cpu().numpy()
        err32 = np.max(np.abs(got32 - ref) / scale)
        say(f"  which={which} fp32 values max rel err={err32:.2e}")
        assert err32 <= 2 * 2.0 ** -24 * 1.01    # one rounding of the value and one of x per product
    sol.close()


# --------------------------------------------------------- whole solves

def test_worked_example_first_iterations():
    """Same closed forms as the oracle pin: exact CG (2 steps, tolerance 0)
    from (0,0); after one iteration x1 = (sqrt2 - 1, 1/(1 + 2 sqrt2))."""
    import math
    import scipy.sparse as sp
    say("[solve] worked example W, 1 iteration")
    qp = I.QP(I.CSR.from_scipy(sp.csr_matrix(np.diag([2.0, 1.0]))), I.CSR.from_scipy(sp.csr_matrix([[1.0, 1.0]])),
              np.array([1.0]), np.array([-2.0, -1.0]))
    x, y, r, _ = gpu_solve(qp, tol_rel_kkt=1e-14, max_iters=1, max_cg_iters=2, cg_eps_factor=0.0, eval_period=1000)
    s2 = math.sqrt(2.0)
    assert r["norm_A"] == pytest.approx(s2, rel=1e-14)
    assert np.allclose(x, [s2 - 1, 1 / (1 + 2 * s2)], atol=1e-14)
    assert y[0] == pytest.approx((2 * (x.sum()) - 1) / (2 * s2), abs=1e-14)
    x, y, r, _ = gpu_solve(qp, tol_rel_kkt=1e-10)
    assert r["status"] == 0
    assert np.allclose(x, [2 / 3, 1 / 3], atol=1e-8)


@pytest.mark.parametrize("inst", range(4))
def test_tiny_case_parity(inst):
    say(f"[solve] random_qp n=1000 m=500 instance={inst}")
    qp = I.random_qp(family=1, instance=inst)
    ref = oracle_ref(qp, ("rq1", inst))
    x, y, r, info = gpu_solve(qp, tol_rel_kkt=1e-6)
    say(f"  status={r['status_name']} iters={r['iters']} cg={r['cg_iters_total']} kkt={r['rel_kkt']:.2e} plan={info}")
    assert r["status"] == 0
    k = check_contract(qp, x, y, ref)
    assert r["rel_kkt"] == pytest.approx(k["rel_kkt"], rel=1e-6, abs=1e-12)


@pytest.mark.parametrize("nb", [1, 3, 8, 64])
def test_grid_sizes(nb):
    """The same solve on 1 (no grid barrier), 3, 8 and 64 workgroups."""
    say(f"[solve] random_qp n=1000 instance=0 num_blocks={nb}")
    qp = I.random_qp(family=1, instance=0)
    ref = oracle_ref(qp, ("rq1", 0))
    x, y, r, info = gpu_solve(qp, tol_rel_kkt=1e-6, num_blocks=nb)
    assert info["num_blocks"] == nb
    assert r["status"] == 0
    check_contract(qp, x, y, ref)


@pytest.mark.parametrize("n,m,inst", [(3, 5, 1), (6, 10, 4), (8, 12, 5)])
def test_brute_force_tiny(n, m, inst):
    say(f"[solve] tiny dense QP n={n} m={m}")
    from test_oracle_pins import brute_force_active_set
    qp = I.tiny_qp(n, m, instance=inst)
    f, xs, ys = brute_force_active_set(qp.Q.to_scipy().toarray(), qp.c, qp.A.to_scipy().toarray(), qp.b)
    x, y, r, _ = gpu_solve(qp, tol_rel_kkt=1e-10, max_iters=400_000)
    assert r["status"] == 0
    assert np.linalg.norm(x - xs) <= 1e-6 * max(1.0, np.linalg.norm(xs))


def test_manufactured_tiny_and_unconstrained():
    say("[solve] manufactured n=1000 m=500")
    qp = I.manufactured()
    x, y, r, _ = gpu_solve(qp, tol_rel_kkt=1e-8)
    assert r["status"] == 0
    assert np.linalg.norm(x - qp.x_star) / np.linalg.norm(qp.x_star) < 1e-5
    say("[solve] unconstrained n=150 (m = 0)")
    qp = I.unconstrained(150)
    xs = -np.linalg.solve(qp.Q.to_scipy().toarray(), qp.c)
    x, y, r, _ = gpu_solve(qp, tol_rel_kkt=1e-10)
    assert r["status"] == 0
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-8


def test_large_case_fp64_and_mixed():
    """n = 1e5, m = 5e4 (R 5e4 x 1e5 at 2e-5, A at 2e-4): FP64 and FP32-product
    solves to relKKT 1e-6 against a manufactured optimum of the same shape and
    against the oracle's KKT of the generated instance."""
    say("[solve] manufactured n=1e5 m=5e4 fp64 and mixed")
    qp = I.manufactured(100_000, 50_000, 2e-5, 2e-4, r_rows=50_000, family=41)
    for prec in (0, 1):
        x, y, r, info = gpu_solve(qp, tol_rel_kkt=1e-6, precision=prec)
        say(f"  precision={prec} status={r['status_name']} iters={r['iters']} cg={r['cg_iters_total']} "
            f"kkt={r['rel_kkt']:.2e} t={r['solve_s']:.3f}s plan={info}")
        assert r["status"] == 0
        k = O.kkt(qp, x, y)
        assert k["rel_kkt"] <= 1e-6 * (1 + 1e-6)
        assert np.linalg.norm(x - qp.x_star) / np.linalg.norm(qp.x_star) < 1e-4
    say("[solve] random_qp n=1e5 m=5e4 mixed, oracle-recomputed KKT")
    qp = I.random_qp(100_000, 50_000, 50_000, 2e-5, 2e-4, family=2)
    x, y, r, info = gpu_solve(qp, tol_rel_kkt=1e-6, precision=1)
    say(f"  status={r['status_name']} iters={r['iters']} cg={r['cg_iters_total']} t={r['solve_s']:.3f}s")
    assert r["status"] == 0
    assert O.kkt(qp, x, y)["rel_kkt"] <= 1e-6 * (1 + 1e-6)


def test_failure_modes_and_limits():
    import scipy.sparse as sp
    say("[solve] NaN in c")
    qp = I.random_qp(family=1, instance=0)
    bad = I.QP(qp.Q, qp.A, qp.b, np.where(np.arange(qp.n) == 3, np.nan, qp.c))
    x, y, r, _ = gpu_solve(bad)
    assert r["status"] == 3
    say("[solve] infeasible pair")
    inf = I.QP(I.CSR.from_scipy(sp.csr_matrix(np.eye(1))), I.CSR.from_scipy(sp.csr_matrix([[1.0], [-1.0]])),
               np.array([-1.0, -1.0]), np.array([0.0]))
    x, y, r, _ = gpu_solve(inf, max_iters=2000)
    assert r["status"] == 1 and r["iters"] == 2000
    say("[solve] iteration cap and time limit")
    x, y, r, _ = gpu_solve(qp, tol_rel_kkt=1e-12, max_iters=10)
    assert r["status"] == 1 and r["iters"] == 10
    x, y, r, _ = gpu_solve(qp, tol_rel_kkt=1e-15, time_limit_s=0.02, max_iters=10**9)
    assert r["status"] == 2 and r["solve_s"] < 5.0
    say("[create] invalid inputs")
    Qd = qp.Q.to_scipy().toarray()
    Qd[0, 1] += 1.0   # not symmetric
    with pytest.raises(pdhcg.PdhcgError) as e:
        pdhcg.Solver(I.QP(I.CSR.from_scipy(sp.csr_matrix(Qd)), qp.A, qp.b, qp.c))
    assert e.value.code == -1
    A = qp.A
    bad_col = I.CSR(A.nrows, A.ncols, A.rowptr, np.where(np.arange(A.nnz) == 5, A.ncols + 3, A.col).astype(np.int32),
                    A.val)
    with pytest.raises(pdhcg.PdhcgError):
        pdhcg.Solver(I.QP(qp.Q, bad_col, qp.b, qp.c))
    unsorted = I.CSR(A.nrows, A.ncols, A.rowptr, A.col.copy(), A.val)
    r0 = int(np.argmax(np.diff(A.rowptr) >= 2))
    a, b_ = A.rowptr[r0], A.rowptr[r0] + 1
    unsorted.col[[a, b_]] = unsorted.col[[b_, a]]
    with pytest.raises(pdhcg.PdhcgError):
        pdhcg.Solver(I.QP(qp.Q, unsorted, qp.b, qp.c))


@pytest.mark.parametrize("precision", [0, 1])
def test_warm_start_resume_negative_y0_and_determinism(precision):
    say(f"[solve] warm start / resume / determinism precision={precision}")
    qp = I.random_qp(family=1, instance=2)
    ref = oracle_ref(qp, ("rq1", 2))
    sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=1e-6, max_iters=200, precision=precision))
    x1, y1, r1 = sol.solve()
    assert r1["status"] == 1
    sol.set_settings(pdhcg.Settings(tol_rel_kkt=1e-6, precision=precision))
    x2, y2, r2 = sol.solve(x0=x1, y0=y1)
    assert r2["status"] == 0
    check_contract(qp, x2.cpu().numpy(), y2.cpu().numpy(), ref)
    # negative y0 is projected: same first iterate as y0 = 0
    sol.set_settings(pdhcg.Settings(tol_rel_kkt=1e-14, max_iters=1, precision=precision))
    xa, _, _ = sol.solve(y0=-np.ones(qp.m))
    xb, _, _ = sol.solve(y0=np.zeros(qp.m))
    assert torch.equal(xa, xb)
    # fixed-order reductions: repeated solves are bit-identical
    sol.set_settings(pdhcg.Settings(tol_rel_kkt=1e-6, precision=precision))
    xa, ya, ra = sol.solve()
    xb, yb, rb = sol.solve()
    assert torch.equal(xa, xb) and torch.equal(ya, yb) and ra["iters"] == rb["iters"]
    sol.close()


@pytest.mark.parametrize("form", [1, 2])
def test_fixed_cg_steps_accounting(form):
    """With a fixed number N of CG steps per iteration (cg_rule 1) every
    iteration takes exactly N steps, whichever code path runs them (in FP32
    products the chained steps hand the last one to the control step)."""
    qp = I.random_qp(family=1, instance=3)
    for n_cg in (2, 3, 7):
        say(f"[solve] random_qp n=1000 instance=3 cg_rule=1 N={n_cg} cg_form={form}")
        x, y, r, _ = gpu_solve(qp, tol_rel_kkt=1e-6, precision=1, cg_rule=1, max_cg_iters=n_cg,
                               max_iters=200_000, cg_form=form)
        assert r["status"] == 0
        assert r["cg_iters_total"] == n_cg * r["iters"]
        assert O.kkt(qp, x, y)["rel_kkt"] <= 1e-6 * (1 + 1e-6)


def test_cg_cap_one_step():
    """CG capped at 1 step (the linearised primal step used as the in-run
    comparison) converges to the same solution, with more iterations."""
    say("[solve] random_qp n=1000 with one CG step per iteration")
    qp = I.random_qp(family=1, instance=1)
    ref = oracle_ref(qp, ("rq1", 1))
    x, y, r, _ = gpu_solve(qp, tol_rel_kkt=1e-6, max_cg_iters=1, cg_rule=1, max_iters=400_000)
    assert r["status"] == 0
    assert r["cg_iters_total"] == r["iters"]
    check_contract(qp, x, y, ref)
    x2, y2, r2, _ = gpu_solve(qp, tol_rel_kkt=1e-6)
    assert r2["iters"] < r["iters"]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("form", [1, 2])
def test_cg_forms(form, precision):
    """Both forms of the CG steps (one reduction per step with (r, u, s)
    gathered, and the textbook form with two) on the same instance and, in
    FP32 products with one tile per workgroup, the chained steps of the first."""
    say(f"[solve] random_qp n=1000 instance=2 cg_form={form} precision={precision}")
    qp = I.random_qp(family=1, instance=2)
    ref = oracle_ref(qp, ("rq1", 2))
    x, y, r, info = gpu_solve(qp, tol_rel_kkt=1e-6, precision=precision, cg_form=form)
    say(f"  status={r['status_name']} iters={r['iters']} cg={r['cg_iters_total']} plan={info}")
    assert r["status"] == 0
    check_contract(qp, x, y, ref)


def test_cg_forms_same_iterates_medium():
    """At n = 2e4 (several workgroups, one CG tile each) the two forms take
    the same iterations up to rounding: equal iteration counts within a few
    and points within the parity bar of each other."""
    say("[solve] random_qp n=20000 m=10000 both CG forms")
    qp = I.random_qp(20_000, 10_000, 10_000, 1e-4, 1e-3, family=2, instance=7)
    out = {}
    for form in (1, 2):
        x, y, r, info = gpu_solve(qp, tol_rel_kkt=1e-6, precision=1, cg_form=form)
        say(f"  form={form} status={r['status_name']} iters={r['iters']} cg={r['cg_iters_total']} plan={info}")
        assert r["status"] == 0
        assert O.kkt(qp, x, y)["rel_kkt"] <= 1e-6 * (1 + 1e-6)
        out[form] = (x, r)
    (x1, r1), (x2, r2) = out[1], out[2]
    assert abs(r1["iters"] - r2["iters"]) <= max(5, r1["iters"] // 20)
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x2) <= 1e-4


def test_powerlaw_parity_small():
    say("[solve] power-law QP n=60000 m=30000 (long rows)")
    qp = I.powerlaw_qp(60_000, 30_000, family=3, instance=1)
    x, y, r, info = gpu_solve(qp, tol_rel_kkt=1e-6, max_iters=200_000)
    say(f"  status={r['status_name']} iters={r['iters']} cg={r['cg_iters_total']} plan={info}")
    assert info["long_rows"] > 0
    assert r["status"] == 0
    assert O.kkt(qp, x, y)["rel_kkt"] <= 1e-6 * (1 + 1e-6)


def test_autotune_then_solve():
    """The autotuner re-plans the partitions; the tuned solve still meets the contract."""
    say("[autotune] random_qp n=1000 instance=3")
    qp = I.random_qp(family=1, instance=3)
    ref = oracle_ref(qp, ("rq1", 3))
    sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=1e-6))
    choice = sol.autotune(iters=20)
    say(f"  chose {choice}")
    assert choice["num_blocks"] in (64, 128, 256, 512) and choice["group_scale"] in (-1, 0, 1)
    assert choice["threads"] in (256, 512) and sol.plan_info()["threads"] == choice["threads"]
    x, y, r = sol.solve()
    assert r["status"] == 0
    check_contract(qp, x.cpu().numpy(), y.cpu().numpy(), ref)
    sol.close()


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("form", [1, 2])
def test_256_thread_workgroups(form, precision):
    """The cooperative kernels compiled for 256-thread workgroups (two per
    CU), forced on a small QP, meet the same contract in both CG forms and
    both precisions."""
    say(f"[solve] random_qp n=1000 instance=2 threads=256 cg_form={form} precision={precision}")
    qp = I.random_qp(family=1, instance=2)
    ref = oracle_ref(qp, ("rq1", 2))
    x, y, r, info = gpu_solve(qp, tol_rel_kkt=1e-6, precision=precision, cg_form=form, threads=256)
    say(f"  status={r['status_name']} iters={r['iters']} cg={r['cg_iters_total']} plan={info}")
    assert info["threads"] == 256
    assert r["status"] == 0
    check_contract(qp, x, y, ref)


def test_256_thread_workgroups_long_rows():
    """256-thread workgroups on the power-law QP with rows longer than a tile."""
    say("[solve] power-law QP n=60000 m=30000 threads=256")
    qp = I.powerlaw_qp(60_000, 30_000, family=3, instance=1)
    x, y, r, info = gpu_solve(qp, tol_rel_kkt=1e-6, max_iters=200_000, threads=256)
    say(f"  status={r['status_name']} iters={r['iters']} cg={r['cg_iters_total']} plan={info}")
    assert info["long_rows"] > 0 and info["threads"] == 256
    assert r["status"] == 0
    assert O.kkt(qp, x, y)["rel_kkt"] <= 1e-6 * (1 + 1e-6)


def test_planner_workgroup_size_and_switch():
    """Past the L2 of one XCD (12 n bytes) the planner takes 256-thread
    workgroups and up to twice the grid; switching to 512 threads through the
    settings re-plans the partitions, and both solves reach the tolerance on
    the FP64 data in nearly the same iterations with nearly the same x."""
    say("[solve] random_qp n=600000 m=300000 planner threads, then 512")
    qp = I.random_qp(600_000, 300_000, 300_000, 5e-6, 3.5e-5, family=2, instance=3)
    sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=1e-5, precision=1))
    out = {}
    try:
        for threads in (0, 512):
            if threads:
                sol.set_settings(pdhcg.Settings(tol_rel_kkt=1e-5, precision=1, threads=threads))
            x, y, r = sol.solve()
            info = sol.plan_info()
            say(f"  threads={threads} status={r['status_name']} iters={r['iters']} plan={info}")
            assert r["status"] == 0
            x, y = x.cpu().numpy(), y.cpu().numpy()
            assert O.kkt(qp, x, y)["rel_kkt"] <= 1e-5 * (1 + 1e-6)
            out[threads] = (x, r, info)
    finally:
        sol.close()
    (x0, r0, i0), (x1, r1, i1) = out[0], out[512]
    assert i0["threads"] == 256 and i1["threads"] == 512
    assert i0["num_blocks"] > 256 >= i1["num_blocks"]
    assert abs(r0["iters"] - r1["iters"]) <= max(64, r1["iters"] // 10)
    assert np.linalg.norm(x0 - x1) / np.linalg.norm(x1) <= 1e-3


def test_autotune_across_workgroup_sizes_large():
    """The autotuner re-plans the partitions of a QP past one XCD's L2 for
    every workgroup size and grid it times (up to 512 workgroups of 256
    threads); the plan it keeps solves to the tolerance on the FP64 data."""
    say("[autotune] random_qp n=300000 m=150000")
    qp = I.random_qp(300_000, 150_000, 150_000, 1e-5, 7e-5, family=2, instance=3)
    sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=1e-5, precision=1))
    try:
        choice = sol.autotune(iters=10)
        info = sol.plan_info()
        say(f"  chose {choice}, plan {info}")
        assert choice["threads"] in (256, 512) and info["threads"] == choice["threads"]
        assert info["num_blocks"] == choice["num_blocks"] <= (512 if choice["threads"] == 256 else 256)
        x, y, r = sol.solve()
        say(f"  status={r['status_name']} iters={r['iters']}")
        assert r["status"] == 0
        assert O.kkt(qp, x.cpu().numpy(), y.cpu().numpy())["rel_kkt"] <= 1e-5 * (1 + 1e-6)
    finally:
        sol.close()


# ----------------------------------------------- full-size power-law (2e6 x 1e6)

def test_powerlaw_full_size_products_and_solve_properties():
    """The power-law configuration at its full size, in the launch configuration
    the benchmark uses (default plan, FP32 products): every product against the
    oracle's FP64 matvec, element by element; a fixed-iteration solve (the
    oracle cannot finish one at this size) checked by properties that hold at
    any size: the reported relKKT equals the oracle's FP64 recomputation at
    the returned point, y >= 0, and a second run is bit-identical."""
    say("[powerlaw full] n=2e6 m=1e6")
    qp = I.powerlaw_qp(2_000_000, 1_000_000, family=3, instance=0)
    sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=1e-12, precision=1, max_iters=40))
    rng = np.random.default_rng(11)
    xn, xm = rng.standard_normal(qp.n), rng.standard_normal(qp.m)
    At = I.CSR.from_scipy(qp.A.to_scipy().T)
    for which, M, v in ((0, qp.Q, xn), (1, qp.A, xn), (2, At, xm)):
        ref = O.matvec(M, v)
        scale = O.matvec(I.CSR(M.nrows, M.ncols, M.rowptr, M.col, np.abs(M.val)), np.abs(v)) + 1e-300
        err = np.max(np.abs(sol.spmv(which, v).cpu().numpy() - ref) / scale)
        err32 = np.max(np.abs(sol.spmv(which, v, precision=1).cpu().numpy() - ref) / scale)
        say(f"  which={which} fp64 {err:.2e} fp32 {err32:.2e}")
        assert err <= 1e-14
        assert err32 <= 2 * 2.0 ** -24 * 1.01
    x1, y1, r1 = sol.solve()
    x1, y1 = x1.cpu().numpy(), y1.cpu().numpy()
    say(f"  40 iterations: relKKT {r1['rel_kkt']:.4e} status {r1['status']}")
    assert r1["status"] == 1 and r1["iters"] == 40
    k = O.kkt(qp, x1, y1)
    assert np.all(y1 >= 0)
    assert abs(k["rel_kkt"] - r1["rel_kkt"]) <= 1e-9 * max(k["rel_kkt"], 1e-300), (k["rel_kkt"], r1["rel_kkt"])
    x2, y2, r2 = sol.solve()
    assert np.array_equal(x1, x2.cpu().numpy()) and np.array_equal(y1, y2.cpu().numpy())
    sol.close()
