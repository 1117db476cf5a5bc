"""Benchmark: time and QPs/s to relKKT <= 1e-4 with restarted PDHCG on one GPU.

Default workload (the largest configuration that fits one GPU; one step = one
batched solve of the whole hot path for every instance: stacked [Q|A'] pass,
inexact CG, projected dual step, averaging, restart evaluation): 4096
portfolio QPs, n log-uniform in [50, 2000], Q = F F' + diag(d) given by its
factor (F n x ceil(n/10), N(0, 1/n)), d ~ U[0.01, 0.1], c = -mu with
mu ~ N(0.05, 0.02^2), rows 1'x <= 1, -1'x <= -1, -x <= 0; diagonal
preconditioning per instance (10 Ruiz steps + Pock-Chambolle, relKKT on each
caller's problem); FP32 products with FP64 reductions; cold start; tol 1e-4.
The batch is generated, packed, uploaded and preconditioned
(pdhcg_batch_create) before the timed region; each timed step is one
pdhcg_batch_solve with device-resident outputs.

Prints one JSON line.  Besides the contract fields it carries the roofline
of the dominant kernel (the batched solve kernel, timed with HIP events on its
own stream), the FP64 CPU oracle timed on this host on a sample of the same
instances, and side measurements (one-by-one solves of a sample, the random
QP n = 1e5, the power-law QP n = 2e6 to 1e-4, learned warm start vs cold).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS_FILE = os.path.join(ROOT, "profiles", "pdhcg_batch_kernel_portfolio_4096_counters.md")
HEADLINE_KERNEL = "pdhcg_batch_kernel"
CALIBRATION_BYTES = 1 << 30   # the --calibrate-copy kernel reads and writes 1 GiB


# the sources that define the solver kernels (single-QP and batched) and how
# they are launched and fed; the network, the standalone product and the
# preconditioning kernels do not run in the measured launches
SOLVER_SOURCES = ["paper_2405_16160_amd/csrc/solve_kernels.hip", "paper_2405_16160_amd/csrc/batch_kernels.hip",
                  "paper_2405_16160_amd/csrc/batch_kernels_512.hip", "paper_2405_16160_amd/csrc/solve_kernels_256.hip",
                  "paper_2405_16160_amd/csrc/solver.hpp", "paper_2405_16160_amd/csrc/device.hpp",
                  "paper_2405_16160_amd/csrc/internal.hpp", "paper_2405_16160_amd/csrc/api.cpp",
                  "include/pdhcg.h"]


def kernel_source_hash():
    """SHA-256 over the sources of the solver kernels and their host side: a
    counter summary is used only while it was measured on the same code."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(os.path.join(ROOT, f) for f in SOLVER_SOURCES)
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def read_counter_csv(d):
    """Per-dispatch counter values (KiB) from a rocprofv3 --pmc CSV run:
    [(kernel_name, counter, value)]."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((r.get("Kernel_Name", ""), r.get("Counter_Name", ""), float(r.get("Counter_Value", 0))))
    return rows


def summarize_counters(d, algorithmic_bytes, kernel=HEADLINE_KERNEL):
    """Scale the kernel's FETCH_SIZE / WRITE_SIZE (KiB per dispatch) by what
    the same counters read for a plain 1 GiB device copy."""
    out = {}
    for counter, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        solve = [v for k, c, v in read_counter_csv(os.path.join(d, sub))
                 if c == counter and kernel in k]
        copy = [v for k, c, v in read_counter_csv(os.path.join(d, "copy_" + sub)) if c == counter]
        if not solve or not copy:
            raise SystemExit(f"no {counter} rows under {d}/{sub} or {d}/copy_{sub}")
        factor = max(copy) * 1024.0 / CALIBRATION_BYTES   # counter bytes per copied byte
        out[counter] = {"solve_kib_per_dispatch": float(np.mean(solve)), "dispatches": len(solve),
                        "copy_kib": max(copy), "factor": factor,
                        "bytes_per_launch": float(np.mean(solve)) * 1024.0 / factor}
    traffic = out["FETCH_SIZE"]["bytes_per_launch"] + out["WRITE_SIZE"]["bytes_per_launch"]
    return {"source_sha256": kernel_source_hash(), "traffic_bytes_per_launch": traffic,
            "algorithmic_bytes_per_launch": algorithmic_bytes, "traffic_over_algorithmic": traffic / algorithmic_bytes,
            "counters": out}


def measured_traffic(path=COUNTERS_FILE):
    """Bytes per launch of a kernel from a committed counter summary (the
    headline kernel's by default), or None when there is none or the sources
    changed since it was taken."""
    if not os.path.exists(path):
        return None, None
    for line in open(path):
        if line.startswith("counters-json: "):
            d = json.loads(line[len("counters-json: "):])
            if d.get("source_sha256") == kernel_source_hash():
                return d["traffic_bytes_per_launch"], d
            return None, None
    return None, None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--precision", type=int, default=1)
    ap.add_argument("--num-blocks", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true", help="skip SpMV and CG-cap-1 side measurements")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (for scaling the FETCH/WRITE counters)")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="turn rocprofv3 --pmc CSV runs under DIR/{fetch,write,copy_fetch,copy_write} into "
                         "the counter summary line (prints it; runs on the CPU)")
    ap.add_argument("--counter-kernel", default=HEADLINE_KERNEL,
                    help="with --summarize-counters: the kernel whose dispatches are summarised")
    ap.add_argument("--bench-line", metavar="FILE",
                    help="with --summarize-counters: a file holding the bench line of the profiled run "
                         "(its algorithmic bytes per launch)")
    ap.add_argument("--config", default="portfolio",
                    choices=["portfolio", "random1e5", "tiny", "powerlaw", "batch", "learned", "kappa", "precondition",
                             "lowrank"],
                    help="workload; the default is the benchmark line, the others are extra measurements")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--threads", type=int, default=0, choices=(0, 256, 512),
                    help="threads per workgroup of the batched kernel (0: the batch autotuner picks)")
    ap.add_argument("--precondition", action="store_true",
                    help="batch mode: 10 Ruiz steps + Pock-Chambolle per instance (no factored run)")
    ap.add_argument("--train", type=int, default=20_000)
    ap.add_argument("--test", type=int, default=4_000)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--iters", type=int, default=300, help="fixed iterations for the power-law bandwidth run")
    return ap.parse_args()


def workload():
    from paper_2405_16160_amd import instances as I
    return I.random_qp(100_000, 50_000, 50_000, 2e-5, 2e-4, family=2, instance=0)


def csr_bytes(nnz, nrows, ncols, sv, sx, sy=None):
    """Compulsory bytes of y = M x: matrix once (values + int32 columns +
    int32 row pointers), x once (sx bytes per entry), y once (sy, default sx)."""
    return nnz * (sv + 4) + 4 * (nrows + 1) + ncols * sx + nrows * (sx if sy is None else sy)


def solve_bytes(qp, r, precision, dense_q=False, rank=0, scaled=False):
    """Algorithmic HBM bytes of one solve, from the counts the solver reports.
    Per iteration: the n-side pass [Q|A'][x;y] in FP64 (r0 and relKKT), the
    dual step y = proj(y + sigma(A(2x+ - x) - b)) with its vectors, and the
    average update; per CG step nnz(Q)(sv+4) + 4(n+1) + 11 n sx (product, dot,
    axpy and direction update with their vectors); per restart evaluation the
    n-side pass and an A product at the average.  For a dense or factored Q
    in the batch the Q part of the n-side pass is counted for the passes that
    formed Q x (qx_formed); the others read the kept Q x.  The n-side pass is FP64 in
    both precision modes by design: it forms r0 and the relKKT pieces, so the
    termination test is taken on the FP64 data.  With preconditioning
    (scaled) every relKKT also reads D2 (n-side) and D1 (m-side)."""
    n, m = qp.n, qp.m
    nq, na = qp.Q.nnz, qp.A.nnz
    sv = sx = 4 if precision == 1 else 8
    dsc = (8 * n + 8 * m) if scaled else 0
    if dense_q:   # a dense Q is stored as n x n values without indices: count it as such
        nq_b64, nq_bv = n * n * 8, n * n * sv
        if rank:  # Q = F F' + diag(d) from its factor: F and F' streamed, d read
            nq_b64, nq_bv = (2 * n * rank + n) * 8, (2 * n * rank + n) * sv
        a1 = na * 12 + 4 * (n + 1) + (n + m) * 8 + 2 * n * 8
        cg = nq_bv + 11 * n * sx
        ev = nq_b64 + na * 12 + 4 * (n + 1) + (n + m) * 8 + n * 8 + csr_bytes(na, m, n, 8, 8) + 2 * m * 8
        dual = csr_bytes(na, m, n, sv, sx) - m * sx + 7 * m * 8 + 3 * n * 8
        # Q x is formed (FP64 product) in qx_formed n-side passes; with Q x
        # kept by linearity the other passes read it (8n) and every CG step
        # updates it (16n)
        formed = r.get("qx_formed", r["iters"])
        kept = formed < r["iters"]
        return (r["iters"] * (a1 + dual + dsc) + formed * nq_b64 + (r["iters"] - formed) * 8 * n * kept
                + r["cg_iters_total"] * (cg + 16 * n * kept) + r["kkt_evals"] * (ev + dsc))
    a1 = (nq + na) * 12 + 8 * (n + 1) + (n + m) * 8 + 2 * n * 8           # matrices, x, y, c, r
    dual = csr_bytes(na, m, n, sv, sx) - m * sx + 7 * m * 8 + 3 * n * 8   # + y, ax, b, ya (r/w); xa update
    cg = nq * (sv + 4) + 4 * (n + 1) + 11 * n * sx
    ev = (nq + na) * 12 + 8 * (n + 1) + (n + m) * 8 + n * 8 + csr_bytes(na, m, n, 8, 8) + 2 * m * 8
    return r["iters"] * (a1 + dual + dsc) + r["cg_iters_total"] * cg + r["kkt_evals"] * (ev + dsc)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_one_core(tol):
    """The same oracle solve on one core: a child process with one OpenMP
    thread (the thread count of a running OpenMP runtime is fixed)."""
    import subprocess
    code = ("import sys, time, json; sys.path.insert(0, %r); "
            "from oracle import oracle as O; from bench import workload; qp = workload(); "
            "t = time.perf_counter(); r = O.solve(qp, O.Settings(tol=%r)); "
            "print(json.dumps({'seconds': time.perf_counter() - t, 'iters': r.iters, "
            "'threads': O.num_threads(), 'status': r.status}))") % (os.path.dirname(os.path.abspath(__file__)), tol)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    progress("oracle solve on one core")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=600)
    if out.returncode != 0:
        return {"error": out.stderr[-500:]}
    d = json.loads(out.stdout.strip().splitlines()[-1])
    d["QPs/s"] = 1.0 / d["seconds"]
    return d


def cpu_baseline(qp, tol):
    """FP64 CPU oracle on this host: one full solve of the same instance to
    the same tolerance (about 3-15 s of CPU work on all cores), and the same
    solve on one core beside it."""
    from oracle import oracle as O
    O.build()
    t = time.perf_counter()
    r = O.solve(qp, O.Settings(tol=tol))
    dt = time.perf_counter() - t
    return {"value": 1.0 / dt, "unit": "QPs/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"one full FP64 solve of the benchmark instance to relKKT <= {tol:g} "
                      f"({r.iters} iterations, {r.cg_steps} CG steps, {dt:.2f} s)",
            "seconds_per_solve": dt, "status": r.status, "cpu_model": cpu_model(),
            "one_core": cpu_one_core(tol)}


def spmv_rates(solver, qp, precisions=(0, 1), reps=50):
    """Standalone product bandwidth: compulsory bytes / kernel time (HIP events)."""
    import torch
    rng = np.random.default_rng(0)
    # x resident on the device before the timed region (no host copy inside it)
    xn = torch.as_tensor(rng.standard_normal(qp.n), device="cuda")
    xm = torch.as_tensor(rng.standard_normal(qp.m), device="cuda")
    out = {}
    for which, name, nnz, nr, nc, v in ((0, "Q", qp.Q.nnz, qp.n, qp.n, xn), (1, "A", qp.A.nnz, qp.m, qp.n, xn),
                                        (2, "At", qp.A.nnz, qp.n, qp.m, xm)):
        for prec in precisions:
            solver.spmv(which, v, precision=prec, repeats=3)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            solver.spmv(which, v, precision=prec, repeats=reps)
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / reps
            sv = 4 if prec else 8   # FP32 mode gathers an FP32 copy of x; y is FP64 either way
            gbs = csr_bytes(nnz, nr, nc, sv, sv, 8) / (us * 1e-6) / 1e9
            out[f"spmv_{name}_{'fp32' if prec else 'fp64'}"] = {"us": us, "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


def spmv_cold_rates(solver, qp, reps=10):
    """Single products with the 256 MB last-level cache (MALL) flushed
    before each: a 1 GiB buffer is written, then one product is timed with
    HIP events (median of reps).  The fill keeps the stream busy long enough
    that the product is queued before its start event is reached.  FP32 times
    include the conversion of x to FP32 (a small extra kernel)."""
    import torch
    rng = np.random.default_rng(0)
    xn = torch.as_tensor(rng.standard_normal(qp.n), device="cuda")
    xm = torch.as_tensor(rng.standard_normal(qp.m), device="cuda")
    flush = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    out = {}
    for which, name, nnz, nr, nc, v in ((0, "Q", qp.Q.nnz, qp.n, qp.n, xn), (1, "A", qp.A.nnz, qp.m, qp.n, xn),
                                        (2, "At", qp.A.nnz, qp.n, qp.m, xm)):
        for prec in (0, 1):
            solver.spmv(which, v, precision=prec, repeats=1)
            ts = []
            for k in range(reps):
                flush.fill_(float(k))
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                solver.spmv(which, v, precision=prec, repeats=1)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e3)
            us = float(np.median(ts))
            sv = 4 if prec else 8
            gbs = csr_bytes(nnz, nr, nc, sv, sv, 8) / (us * 1e-6) / 1e9
            out[f"spmv_{name}_{'fp32' if prec else 'fp64'}"] = {"us": us, "GB/s": gbs, "frac": gbs / HBM_PEAK_GBS}
    del flush
    return out


def instances_geomean(args, count=10):
    """Time to tolerance on instances 0..count-1 of the benchmark family:
    one warm-up and args.steps timed solves each (median), geometric mean
    over the instances."""
    import torch
    from paper_2405_16160_amd import instances as I, pdhcg
    times, iters, cg = [], [], []
    for inst in range(count):
        qp = I.random_qp(100_000, 50_000, 50_000, 2e-5, 2e-4, family=2, instance=inst)
        sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=args.tol, precision=args.precision,
                                              num_blocks=args.num_blocks))
        sol.solve()
        ts = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, _, r = sol.solve()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
            assert r["status"] == 0, r["status_name"]
        times.append(float(np.median(ts)))
        iters.append(r["iters"])
        cg.append(r["cg_iters_total"])
        sol.close()
        progress(f"instance {inst}: {times[-1] * 1e3:.1f} ms, {iters[-1]} iterations")
    g = float(np.exp(np.mean(np.log(times))))
    return {"instances": count, "geomean_ms": g * 1e3, "QPs/s": 1.0 / g,
            "ms": [t * 1e3 for t in times], "iters": iters, "cg_steps": cg}


def bench_tiny(args):
    """n = 1000, m = 500 FP64 random QP, 10 instances, tol 1e-4."""
    import torch
    from paper_2405_16160_amd import instances as I, pdhcg
    times, iters = [], []
    for inst in range(10):
        qp = I.random_qp(family=1, instance=inst)
        sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=args.tol, num_blocks=args.num_blocks))
        sol.solve()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            _, _, r = sol.solve()
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t) / args.steps)
        iters.append(r["iters"])
        plan = sol.plan_info()
        sol.close()
    g = float(np.exp(np.mean(np.log(times))))
    return {"config": "tiny random QP n=1000 m=500 FP64, 10 instances, tol %g" % args.tol,
            "geomean_ms": g * 1e3, "QPs/s": 1 / g, "iters": iters, "plan": plan}


def local_columns_rates(qp):
    """The power-law A with the same row lengths but each row's columns a
    contiguous block near its diagonal position (gathers coalesce and x stays
    in cache): separates the product's streaming rate from the cost of the
    random gathers of the benchmark matrix."""
    from paper_2405_16160_amd import instances as I, pdhcg
    m, n = qp.A.nrows, qp.A.ncols
    lens = np.diff(qp.A.rowptr)
    centre = (np.arange(m, dtype=np.int64) * n) // m
    start = np.clip(centre - lens // 2, 0, n - lens)
    rowptr = qp.A.rowptr.astype(np.int64)
    col = (np.repeat(start, lens) + (np.arange(rowptr[-1]) - np.repeat(rowptr[:-1], lens))).astype(np.int32)
    A = I.CSR(m, n, rowptr, col, qp.A.val.copy())
    Qd = I.CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.ones(n))
    loc = I.QP(Qd, A, qp.b, qp.c)
    sol = pdhcg.Solver(loc, pdhcg.Settings(precision=1))
    r = spmv_rates(sol, loc)
    sol.close()
    return {k: v for k, v in r.items() if not k.startswith("spmv_Q")}


def bench_powerlaw(args):
    """n = 2e6, m = 1e6 power-law QP: standalone products and a fixed number
    of solve iterations (bandwidth of the phases; the family converges slowly
    without preconditioning, so time-to-tolerance is not measured here)."""
    import torch
    from paper_2405_16160_amd import instances as I, pdhcg
    t = time.perf_counter()
    qp = I.powerlaw_qp(2_000_000, 1_000_000, family=3, instance=0)
    gen_s = time.perf_counter() - t
    lens = np.diff(qp.A.rowptr)
    sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=1e-12, precision=args.precision, max_iters=args.iters,
                                          num_blocks=args.num_blocks))
    rates = spmv_rates(sol, qp)
    cold = spmv_cold_rates(sol, qp)
    local = local_columns_rates(qp)
    sol.solve()
    torch.cuda.synchronize()
    _, _, r = sol.solve()
    bytes_alg = solve_bytes(qp, r, args.precision)
    ach = bytes_alg / r["kernel_s"] / 1e9
    out = {"config": "power-law QP n=2e6 m=1e6 (A row lengths Pareto 1.5, mean 8, max 5000)",
           "nnz_Q": qp.Q.nnz, "nnz_A": qp.A.nnz, "A_row_max": int(lens.max()), "gen_s": gen_s,
           "plan": sol.plan_info(), "spmv": rates, "spmv_cold": cold, "spmv_local_columns": local,
           "solve_fixed_iters": {"iters": r["iters"], "cg_steps": r["cg_iters_total"], "kernel_ms": r["kernel_s"] * 1e3,
                                 "us_per_iter": r["kernel_s"] * 1e6 / max(r["iters"], 1), "rel_kkt": r["rel_kkt"],
                                 "GB/s": ach, "frac": ach / HBM_PEAK_GBS}}
    sol.close()
    return out


def progress(msg):
    """A progress line on stderr (long modes), so a watcher sees the run advance."""
    print(f"[bench] {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def bench_batch(args):
    """4096 portfolio QPs (n log-uniform in [50, 2000], dense Q = FF' + D) in one
    batched solve, then the same QPs with Q given by its factor, against
    one-by-one solves of a stratified sample (kernel seconds against kernel
    seconds).  --precondition scales every instance (dense and factored)."""
    import threading
    from paper_2405_16160_amd import instances as I, pdhcg
    t = time.perf_counter()
    qps = []
    for i in range(args.batch_count):
        qps.append(I.portfolio_qp(i))
        if (i + 1) % 256 == 0:
            progress(f"generated {i + 1} portfolio QPs")
    gen_s = time.perf_counter() - t
    pre = {"ruiz_iters": 10, "pock_chambolle": 1} if args.precondition else {}
    s = pdhcg.Settings(tol_rel_kkt=args.tol, precision=args.precision, max_iters=200_000, **pre)
    t = time.perf_counter()
    done = threading.Event()

    def ticker():   # the batched solve is one call; report that it is still running
        while not done.wait(30.0):
            progress(f"batched solve running ({time.perf_counter() - t:.0f} s)")

    th = threading.Thread(target=ticker, daemon=True)
    th.start()
    try:
        out = pdhcg.solve_batch(qps, s)
    finally:
        done.set()
        th.join()
    wall = time.perf_counter() - t
    progress(f"batched solve done in {wall:.1f} s; one-by-one sample")
    rs = [o[2] for o in out]
    ok = sum(r["status"] == 0 for r in rs)
    kernel_s = rs[0]["kernel_s"]
    setup_s = rs[0]["setup_s"]
    # one-by-one baseline on a stratified sample: 2 instances per log-size bin
    ns = np.array([q.n for q in qps])
    edges = np.exp(np.linspace(np.log(50), np.log(2000), 17))
    sample, weights = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        idx = np.nonzero((ns >= a) & (ns < b + 1e-9))[0]
        if idx.size:
            pick = idx[:2]
            sample += list(pick)
            weights += [idx.size / pick.size] * pick.size
    single_s = 0.0
    for i, w in zip(sample, weights):
        sol = pdhcg.Solver(qps[i], s)
        _, _, r = sol.solve()
        single_s += w * r["kernel_s"]
        sol.close()
        progress(f"one-by-one instance {i} (n={qps[i].n}): {r['kernel_s']:.3f} s of kernel time")
    alg = sum(solve_bytes(q, r, args.precision, dense_q=True, scaled=bool(pre)) for q, r in zip(qps, rs))
    # the same QPs with Q given by its factor (Q = F F' + diag(d), k = ceil(n/10))
    progress("factored form: generating the factors")
    fac = [I.portfolio_factor(i) for i in range(args.batch_count)]
    t = time.perf_counter()
    out_lr = pdhcg.solve_batch(qps, s, lowrank=fac)
    wall_lr = time.perf_counter() - t
    rs_lr = [o[2] for o in out_lr]
    kernel_lr = rs_lr[0]["kernel_s"]
    alg_lr = sum(solve_bytes(q, r, args.precision, dense_q=True, rank=f[0].shape[1], scaled=bool(pre))
                 for q, r, f in zip(qps, rs_lr, fac))
    progress(f"factored batch done in {wall_lr:.1f} s")
    lowrank = {"solved": sum(r["status"] == 0 for r in rs_lr), "batch_kernel_s": kernel_lr, "batch_wall_s": wall_lr,
               "QPs/s_batched": args.batch_count / kernel_lr, "iters_mean": float(np.mean([r["iters"] for r in rs_lr])),
               "roofline": {"kernel": "pdhcg_batch_kernel", "bound": "hbm", "algorithmic_bytes": alg_lr,
                            "achieved": alg_lr / kernel_lr / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": alg_lr / kernel_lr / 1e9 / HBM_PEAK_GBS},
               "speedup_vs_dense_batch": kernel_s / kernel_lr, "speedup_vs_one_by_one": single_s / kernel_lr}
    return {"config": f"batched portfolio QPs x{args.batch_count}, n log-uniform [50, 2000], dense Q, tol {args.tol:g}"
                      + (", 10 Ruiz steps + Pock-Chambolle per instance" if pre else ""),
            "lowrank": lowrank,
            "solved": ok, "batch_kernel_s": kernel_s, "batch_wall_s": wall, "setup_s": setup_s,
            "roofline": {"kernel": "pdhcg_batch_kernel", "bound": "hbm", "algorithmic_bytes": alg,
                         "achieved": alg / kernel_s / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": alg / kernel_s / 1e9 / HBM_PEAK_GBS},
            "QPs/s_batched": args.batch_count / kernel_s, "gen_s": gen_s,
            "iters_mean": float(np.mean([r["iters"] for r in rs])),
            "one_by_one_estimated_s": single_s, "QPs/s_one_by_one": args.batch_count / single_s,
            "one_by_one_sample": len(sample), "speedup": single_s / kernel_s}


def bench_kappa(args):
    """Condition sweep (the shape of Table 2): n = m = 5e4, A at density 1e-3,
    Q with condition number kappa in 1 .. 1e5 (kappa_qp).  PDHCG (adaptive CG)
    against CG capped at one step (the linearised primal step), each to tol,
    the capped runs bounded by a 20 s time limit."""
    import torch
    from paper_2405_16160_amd import instances as I, pdhcg
    rows = []
    for kappa in (1.0, 1e1, 1e2, 1e3, 1e4, 1e5):
        qp = I.kappa_qp(kappa)
        row = {"kappa": kappa}
        for name, extra in (("pdhcg", {}), ("cg_cap_1", {"max_cg_iters": 1, "cg_rule": 1})):
            st = pdhcg.Settings(tol_rel_kkt=args.tol, precision=args.precision, max_iters=1_000_000,
                                time_limit_s=20.0, **extra)
            sol = pdhcg.Solver(qp, st)
            _, _, r = sol.solve()
            torch.cuda.synchronize()
            sol.close()
            row[name] = {"status": r["status_name"], "iters": r["iters"], "cg_steps": r["cg_iters_total"],
                         "kernel_ms": r["kernel_s"] * 1e3, "rel_kkt": r["rel_kkt"]}
            progress(f"kappa {kappa:g} {name}: {r['status_name']} {r['iters']} iterations, "
                     f"{r['cg_iters_total']} CG steps, {r['kernel_s'] * 1e3:.1f} ms")
        rows.append(row)
    return {"config": f"condition sweep, kappa_qp n=m=5e4, A density 1e-3, tol {args.tol:g}, "
                      f"precision {args.precision}", "rows": rows}


def bench_lowrank(args):
    """Low-rank Q (the experiment of Tables 3 and 4: Q = P P' with growing
    rank k, each product with Q formed as P (P' v) against the explicit Q):
    lowrank_qp n = 1e5, m = 5e4, P at density 1e-3 (plus d ~ U[0.01, 0.1]),
    k in 1e3 .. 1e4, solved to tol by PDHCG and by CG capped at one step (the
    linearised primal step), each with Q in low-rank form
    (pdhcg_create_lowrank) and explicit (pdhcg_create), kernel time from the
    HIP events of each solve; ratio = low-rank / explicit."""
    import torch
    from paper_2405_16160_amd import instances as I, pdhcg
    rows = []
    for k in (1_000, 2_000, 5_000, 10_000):
        qp, P, d = I.lowrank_qp(n=100_000, m=50_000, k=k)
        row = {"k": k, "nnz_P": P.nnz, "nnz_Q": qp.Q.nnz}
        for name, extra in (("pdhcg", {}), ("cg_cap_1", {"max_cg_iters": 1, "cg_rule": 1})):
            out = {}
            for form, lr in (("low_rank", (P, d)), ("explicit", None)):
                st = pdhcg.Settings(tol_rel_kkt=args.tol, precision=args.precision, max_iters=1_000_000,
                                    time_limit_s=30.0, **extra)
                sol = pdhcg.Solver(qp, st, lowrank=lr)
                _, _, r = sol.solve()
                torch.cuda.synchronize()
                sol.close()
                out[form] = {"status": r["status_name"], "iters": r["iters"], "cg_steps": r["cg_iters_total"],
                             "kernel_ms": r["kernel_s"] * 1e3}
                progress(f"k {k} {name} {form}: {r['status_name']} {r['iters']} iterations, "
                         f"{r['cg_iters_total']} CG steps, {r['kernel_s'] * 1e3:.1f} ms")
            out["ratio"] = out["low_rank"]["kernel_ms"] / out["explicit"]["kernel_ms"]
            row[name] = out
        rows.append(row)
    return {"config": f"low-rank Q, lowrank_qp n=1e5 m=5e4, P density 1e-3, tol {args.tol:g}, "
                      f"precision {args.precision}", "rows": rows}


def bench_precondition(args):
    """Diagonal preconditioning (10 Ruiz steps + one Pock-Chambolle step on
    [[Q, A'], [A, 0]]): the random QP n = 1e5 as generated and with its rows of
    A (and b) rescaled by exp(U[-3, 3]), each solved to tol without and with
    the preconditioning; the power-law QP n = 2e6 for the cost of the setup
    kernels and a time-limited solve; portfolio instances 0-15 one by one.  relKKT
    always refers to the caller's problem; x_rel_diff compares the returned x
    with the unpreconditioned solve's."""
    import torch
    from paper_2405_16160_amd import instances as I, pdhcg
    rows = []
    cases = [("random_qp n=1e5", lambda: I.random_qp(100_000, 50_000, 50_000, 2e-5, 2e-4, family=2), None),
             ("random_qp n=1e5, rows x exp(U[-3,3])",
              lambda: I.row_scaled(I.random_qp(100_000, 50_000, 50_000, 2e-5, 2e-4, family=2)), None),
             ("powerlaw_qp n=2e6", lambda: I.powerlaw_qp(), 15.0)]
    for name, make, tl in cases:
        qp = make()
        row = {"workload": name}
        xs = {}
        for tag, pre in (("plain", {}), ("preconditioned", {"ruiz_iters": 10, "pock_chambolle": 1})):
            st = pdhcg.Settings(tol_rel_kkt=args.tol, precision=args.precision, time_limit_s=tl or 0.0, **pre)
            t0 = time.perf_counter()
            sol = pdhcg.Solver(qp, st)
            torch.cuda.synchronize()
            create_s = time.perf_counter() - t0
            x, _, r = sol.solve()
            torch.cuda.synchronize()
            xs[tag] = x.clone()
            sol.close()
            row[tag] = {"status": r["status_name"], "iters": r["iters"], "cg_steps": r["cg_iters_total"],
                        "kernel_ms": r["kernel_s"] * 1e3, "rel_kkt": r["rel_kkt"], "create_s": create_s,
                        "primal_obj": r["primal_obj"]}
            progress(f"{name} {tag}: {r['status_name']} {r['iters']} iterations, {r['cg_iters_total']} CG steps, "
                     f"{r['kernel_s'] * 1e3:.1f} ms, create {create_s:.2f} s")
        row["x_rel_diff"] = float(torch.linalg.norm(xs["preconditioned"] - xs["plain"]) /
                                  torch.linalg.norm(xs["plain"]))
        rows.append(row)
    # portfolio instances 0-15 (n log-uniform in [50, 2000], dense Q as CSR), one single-QP solve each
    port = {"workload": "portfolio_qp instances 0-15, single-QP solves"}
    qps = [I.portfolio_qp(i) for i in range(16)]
    for tag, pre in (("plain", {}), ("preconditioned", {"ruiz_iters": 10, "pock_chambolle": 1})):
        tot_ms, tot_it, solved = 0.0, 0, 0
        for qp in qps:
            sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=args.tol, precision=args.precision, **pre))
            _, _, r = sol.solve()
            sol.close()
            tot_ms += r["kernel_s"] * 1e3
            tot_it += r["iters"]
            solved += r["status"] == 0
        port[tag] = {"kernel_ms_total": tot_ms, "iters_total": tot_it, "solved": solved}
        progress(f"portfolio 0-15 {tag}: {solved}/16 solved, {tot_it} iterations, {tot_ms:.1f} ms")
    port["n"] = [q.n for q in qps]
    rows.append(port)
    return {"config": f"preconditioning, tol {args.tol:g}, precision {args.precision}", "rows": rows}


def stream_ceiling(gib=2, reps=5):
    """The device's practical streaming rate on this run's GPU, for scale next
    to the roofline's nominal 8 TB/s: a device copy of `gib` GiB (torch's copy
    kernel, timed with events, the best of `reps`; it reads and writes its size
    once each)."""
    import torch
    a = torch.ones((gib << 30) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    out = {"copy_GBps": 2 * a.numel() * 4 / best / 1e9}
    del a, b
    torch.cuda.empty_cache()
    return out


def held_out_solves(fam, ids, settings, starts):
    """Batched solves of the family members `ids` from each start in `starts`
    (pairs of packed float64 device tensors or None), one packed batch;
    returns [(results, kernel seconds)] in the order of `starts`."""
    from paper_2405_16160_amd import pdhcg, warmstart as W
    _, qps = W.family_qps(fam, ids)
    b = pdhcg.Batch(qps, settings)
    out = []
    for x0, y0 in starts:
        _, _, rs = b.solve(x0=None if x0 is None else x0.reshape(-1), y0=None if y0 is None else y0.reshape(-1))
        out.append((rs, rs[0]["kernel_s"]))
    b.close()
    return out


def bench_learned(args):
    """Learned warm start on the MPC family: train on PDHCG solutions, then
    batched cold vs warm solves of held-out members to tol.  The start points
    are predicted and decoded on the device and handed to the batch there."""
    import dataclasses
    from paper_2405_16160_amd import instances as I, pdhcg, warmstart as W
    fam = I.mpc_family()
    plus, minus = W.pair_index(fam)
    progress(f"solving {args.train} training QPs")
    th, X, Y, rs, gen_solve_s = W.solve_family(fam, range(args.train), pdhcg.Settings(tol_rel_kkt=1e-6),
                                               log=progress)
    Y = W.canonical_duals(Y, plus, minus)
    t_train = time.perf_counter()
    progress("training")
    ws, losses = W.train(th, X, Y, W.DualCode(fam.A.nrows, plus, minus), epochs=args.epochs,
                         log=lambda m: progress(m) if int(m.split()[1].rstrip(":")) % 50 == 0 else None)
    train_s = time.perf_counter() - t_train
    ids = range(100_000, 100_000 + args.test)
    th_t, _ = W.family_qps(fam, ids)
    import torch
    t = time.perf_counter()
    x0, y0 = ws.predict_device(th_t)
    torch.cuda.synchronize()
    infer_s = time.perf_counter() - t
    s = pdhcg.Settings(tol_rel_kkt=args.tol, warm_fallback=0)
    (rc, tc), (rw, tw), (rx, tx) = held_out_solves(fam, ids, s, [(None, None), (x0, y0), (x0, None)])
    ((rf, tf),) = held_out_solves(fam, ids, dataclasses.replace(s, warm_fallback=1), [(x0, y0)])
    # single-QP mode on a sample: one handle for the family (Q, A, c shared), b
    # replaced per member, cold and warm solves with the cooperative kernel
    n_single = min(200, args.test)
    _, qps_s = W.family_qps(fam, list(ids)[:n_single])
    sol = pdhcg.Solver(qps_s[0], s)
    single = {"cold": [0.0, 0], "warm": [0.0, 0]}
    progress(f"single-QP solves of {n_single} held-out members, cold and warm")
    for k, q in enumerate(qps_s):
        sol.set_b(q.b)
        for mode, start in (("cold", (None, None)), ("warm", (x0[k], y0[k]))):
            _, _, r = sol.solve(x0=start[0], y0=start[1])
            assert r["status"] == 0, r["status_name"]
            single[mode][0] += r["kernel_s"]
            single[mode][1] += r["iters"]
    sol.close()
    single_row = {m: {"kernel_s": v[0], "QPs/s": n_single / v[0], "iters_mean": v[1] / n_single}
                  for m, v in single.items()}
    single_row["speedup_warm_vs_cold"] = single["cold"][0] / single["warm"][0]
    single_row["sample"] = n_single

    def row(r, secs):
        return {"kernel_s": secs, "QPs/s": args.test / secs, "iters_mean": float(np.mean([x["iters"] for x in r])),
                "solved": sum(x["status"] == 0 for x in r)}

    fb = row(rf, tf)
    fb["fallback_rate"] = float(np.mean([x["cold_fallback"] for x in rf]))
    return {"config": f"learned warm start, MPC T=50 (n=1500, m=5000), train {args.train}, "
                      f"epochs {args.epochs}, test {args.test}, tol {args.tol:g}",
            "train_solves_s": gen_solve_s, "train_s": train_s, "loss_first_last": [losses[0], losses[-1]],
            "infer_s": infer_s, "cold": row(rc, tc), "warm": row(rw, tw),
            "warm_per_instance_fallback": fb, "warm_primal_only": row(rx, tx), "single_qp": single_row,
            "speedup_warm_vs_cold": tc / tw, "speedup_warm_vs_cold_incl_inference": tc / (tw + infer_s)}


PRE = {"ruiz_iters": 10, "pock_chambolle": 1}
HEADLINE_WORKLOAD = ("4096 portfolio QPs batched, n log-uniform [50, 2000], Q = FF' + diag(d) as its factor "
                     "(k = ceil(n/10)), rows 1'x<=1, -1'x<=-1, -x<=0; per-instance Ruiz(10) + Pock-Chambolle "
                     "preconditioning, relKKT on each caller's problem; FP32 products + FP64 reductions; "
                     "cold start; tol 1e-4")


def portfolio_set(count):
    """The headline instances in factored form: [(qp, (F, d))]."""
    from paper_2405_16160_amd import instances as I
    out = []
    for i in range(count):
        out.append(I.portfolio_lowrank(i))
        if (i + 1) % 1024 == 0:
            progress(f"generated {i + 1} portfolio QPs")
    return out


def _oracle_worker(job):
    """One oracle solve of a portfolio instance in a worker pinned to one core
    (single-threaded oracle): the preprocessing and the FP64 solve of the
    oracle package, on the dense Q, to tol.  Returns seconds."""
    core, inst, tol = job
    os.sched_setaffinity(0, {core})
    from oracle import oracle as O, precondition as P
    from paper_2405_16160_amd import instances as I
    qp = I.portfolio_qp(inst)
    t = time.perf_counter()
    _, _, r, _, _ = P.solve(qp, O.Settings(tol=tol, max_iters=400_000))
    return time.perf_counter() - t, r.status, qp.n


def cpu_baseline_portfolio(count, tol, stride=32):
    """The FP64 oracle on this host's cores over a sample of the headline
    instances (every stride-th id, which has the same size distribution):
    instances spread over single-threaded worker processes, one per core and
    pinned to it, as QPs/s of the sample (instances / wall seconds)."""
    import multiprocessing as mp
    from oracle import oracle as O
    O.build()
    cores = sorted(os.sched_getaffinity(0))[:16]
    ids = list(range(0, count, stride))
    jobs = [(cores[k % len(cores)], i, tol) for k, i in enumerate(ids)]
    progress(f"CPU oracle: {len(ids)} portfolio instances on {len(cores)} pinned single-threaded workers")
    env_old = os.environ.get("OMP_NUM_THREADS")
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        ctx = mp.get_context("spawn")
        t = time.perf_counter()
        with ctx.Pool(len(cores)) as pool:
            res = pool.map(_oracle_worker, jobs, chunksize=1)
        wall = time.perf_counter() - t
    finally:
        if env_old is None:
            os.environ.pop("OMP_NUM_THREADS", None)
        else:
            os.environ["OMP_NUM_THREADS"] = env_old
    secs = [r[0] for r in res]
    return {"value": len(ids) / wall, "unit": "QPs/s", "cores": len(cores), "kind": "oracle",
            "sample": f"{len(ids)} of the {count} portfolio instances (ids 0, {stride}, ..., dense Q, the oracle's "
                      f"Ruiz + Pock-Chambolle preprocessing and FP64 solve to relKKT <= {tol:g}), one "
                      f"single-threaded worker process per pinned core; {wall:.1f} s wall",
            "wall_s": wall, "cpu_s_total": float(sum(secs)), "solved": sum(r[1] == 0 for r in res),
            "cpu_model": cpu_model()}


def one_by_one_sample(pairs, args, per_bin=2):
    """Single-QP solves (pdhcg_solve, cooperative kernel, preconditioned, dense
    Q as CSR) of a stratified sample: per_bin instances per log-size bin,
    weighted by the bin's count; kernel seconds against kernel seconds."""
    from paper_2405_16160_amd import instances as I, pdhcg
    ns = np.array([q.n for q, _ in pairs])
    edges = np.exp(np.linspace(np.log(50), np.log(2000), 17))
    est, sample = 0.0, 0
    s = pdhcg.Settings(tol_rel_kkt=args.tol, precision=args.precision, max_iters=200_000, **PRE)
    for a, b in zip(edges[:-1], edges[1:]):
        idx = np.nonzero((ns >= a) & (ns < b + 1e-9))[0]
        if not idx.size:
            continue
        pick = idx[:per_bin]
        for i in pick:
            sol = pdhcg.Solver(I.portfolio_qp(int(i)), s)
            _, _, r = sol.solve()
            sol.close()
            est += (idx.size / pick.size) * r["kernel_s"]
            sample += 1
    progress(f"one-by-one sample of {sample}: estimated {est:.2f} s of kernel time for all")
    return {"sample": sample, "estimated_kernel_s_all": est, "QPs/s": len(pairs) / est}


def side_random1e5(args):
    """The random sparse QP n = 1e5 (plain, cold, FP32 products): kernel ms
    and QPs/s over args.steps solves, and CG capped at one step beside it."""
    import torch
    from paper_2405_16160_amd import pdhcg
    qp = workload()
    sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=args.tol, precision=1))
    sol.solve()
    torch.cuda.synchronize()
    t = time.perf_counter()
    ks = []
    for _ in range(5):
        _, _, r = sol.solve()
        ks.append(r["kernel_s"])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / 5
    sol.set_settings(pdhcg.Settings(tol_rel_kkt=args.tol, precision=1, max_cg_iters=1, cg_rule=1, max_iters=200_000))
    _, _, r1 = sol.solve()
    sol.close()
    return {"workload": "random sparse QP n=1e5 m=5e4, plain, FP32 products, cold, tol 1e-4",
            "QPs/s": 1.0 / dt, "ms_per_solve": dt * 1e3, "kernel_ms": float(np.mean(ks)) * 1e3,
            "iters": r["iters"], "cg_steps": r["cg_iters_total"], "status": r["status_name"],
            "cg_cap_1": {"iters": r1["iters"], "kernel_ms": r1["kernel_s"] * 1e3, "status": r1["status_name"]}}


def side_powerlaw(args):
    """The power-law QP n = 2e6, m = 1e6 to relKKT 1e-4 on its own problem
    (preconditioned, FP32 products): time to tolerance."""
    import torch
    from paper_2405_16160_amd import instances as I, pdhcg
    qp = I.powerlaw_qp()
    t = time.perf_counter()
    sol = pdhcg.Solver(qp, pdhcg.Settings(tol_rel_kkt=args.tol, precision=1, time_limit_s=30.0, **PRE))
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t
    _, _, r = sol.solve()
    sol.close()
    return {"workload": "power-law QP n=2e6 m=1e6, preconditioned, FP32 products, cold, tol 1e-4",
            "status": r["status_name"], "kernel_ms": r["kernel_s"] * 1e3, "solve_ms": r["solve_s"] * 1e3,
            "iters": r["iters"], "cg_steps": r["cg_iters_total"], "rel_kkt": r["rel_kkt"], "create_s": create_s}


def side_warm_start(args, train=4096, test=1024, epochs=60):
    """Learned warm start on the MPC family at a reduced size (train solves,
    epochs and held-out instances below the configuration's 100k / 10k):
    batched cold vs warm kernel time on the held-out instances, inference
    included in the second ratio."""
    from paper_2405_16160_amd import instances as I, pdhcg, warmstart as W
    fam = I.mpc_family()
    plus, minus = W.pair_index(fam)
    th, X, Y, _, gen_s = W.solve_family(fam, range(train), pdhcg.Settings(tol_rel_kkt=1e-6))
    Y = W.canonical_duals(Y, plus, minus)
    t = time.perf_counter()
    ws, losses = W.train(th, X, Y, W.DualCode(fam.A.nrows, plus, minus), epochs=epochs)
    train_s = time.perf_counter() - t
    ids = range(100_000, 100_000 + test)
    th_t, _ = W.family_qps(fam, ids)
    import torch
    t = time.perf_counter()
    x0, y0 = ws.predict_device(th_t)
    torch.cuda.synchronize()
    infer_s = time.perf_counter() - t
    ws.net.close()
    s = pdhcg.Settings(tol_rel_kkt=args.tol, warm_fallback=0)
    (rc, tc), (rw, tw) = held_out_solves(fam, ids, s, [(None, None), (x0, y0)])
    progress(f"warm start: cold {tc:.3f} s, warm {tw:.3f} s, inference {infer_s:.3f} s")
    return {"workload": f"MPC T=50 (n=1500, m=5000), reduced: {train} training solves, {epochs} epochs, "
                        f"{test} held-out, batched, tol {args.tol:g}",
            "cold_kernel_s": tc, "warm_kernel_s": tw, "infer_s": infer_s, "train_s": train_s,
            "cold_iters_mean": float(np.mean([r["iters"] for r in rc])),
            "warm_iters_mean": float(np.mean([r["iters"] for r in rw])),
            "speedup_warm_vs_cold": tc / tw, "speedup_incl_inference": tc / (tw + infer_s),
            "solved": [sum(r["status"] == 0 for r in rc), sum(r["status"] == 0 for r in rw)]}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); "
              "the solver does not shard a QP across GPUs.", file=sys.stderr)
        sys.exit(2)
    if args.summarize_counters:
        line = [json.loads(x) for x in open(args.bench_line) if x.startswith('{"metric"')][-1]
        alg = line["roofline"]["algorithmic_bytes_per_launch"]
        print("counters-json: " + json.dumps(summarize_counters(args.summarize_counters, alg, args.counter_kernel)))
        return
    import torch
    from paper_2405_16160_amd import pdhcg
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        # a copy moves its size twice (read + write): the device's practical streaming rate
        print(json.dumps({"calibrate_copy_bytes": a.numel() * 8, "copies": 3, "ms_per_copy": ms,
                          "copy_GB/s_read_plus_write": 2 * a.numel() * 8 / (ms * 1e-3) / 1e9}))
        return

    if args.config not in ("portfolio", "random1e5"):
        line = {"tiny": bench_tiny, "powerlaw": bench_powerlaw, "batch": bench_batch, "kappa": bench_kappa,
                "precondition": bench_precondition, "learned": bench_learned,
                "lowrank": bench_lowrank}[args.config](args)
        print(json.dumps(line), flush=True)
        return
    if args.config == "random1e5":
        bench_random1e5(args)
        return

    # ---- headline: the batched portfolio configuration
    count = args.batch_count
    pairs = portfolio_set(count)
    qps, facs = [q for q, _ in pairs], [f for _, f in pairs]
    settings = pdhcg.Settings(tol_rel_kkt=args.tol, precision=args.precision, max_iters=200_000, **PRE)
    t = time.perf_counter()
    batch = pdhcg.Batch(qps, settings, lowrank=facs)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t
    progress(f"batch created in {create_s:.2f} s (pack, upload, preconditioning)")
    if args.threads:
        batch.set_threads(args.threads)
        tuned = {"threads": args.threads}
    else:  # untimed set-up: one cold solve of the batch per workgroup size
        tuned = batch.autotune(reps=1)
        progress(f"autotuner: {tuned}")
    kernel_name = HEADLINE_KERNEL if batch.threads == 256 else HEADLINE_KERNEL + "_wg512"
    for _ in range(args.warmup):
        batch.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for _ in range(args.steps):
        _, _, rs = batch.solve()
        runs.append(rs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rs = runs[-1]
    solved = sum(r["status"] == 0 for r in rs)
    assert all(r["status"] == 0 for run in runs for r in run), "an instance did not reach the tolerance"
    kernel_s = float(np.mean([run[0]["kernel_s"] for run in runs]))   # one launch per batched solve
    bytes_alg = sum(solve_bytes(q, r, args.precision, dense_q=True, rank=f[0].shape[1], scaled=True)
                    for q, r, f in zip(qps, rs, facs))
    achieved = bytes_alg / kernel_s / 1e9
    traffic, _ = measured_traffic() if kernel_name == HEADLINE_KERNEL else (None, None)
    progress(f"{args.steps} batched solves: {dt / args.steps:.3f} s each, kernel {kernel_s:.3f} s")
    line = {
        "metric": "time & QPs/s to rel. KKT<=1e-4 (batched/warm-start vs plain); SpMV HBM GB/s",
        "value": count * args.steps / dt,
        "unit": "QPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": HEADLINE_WORKLOAD, "instances": count, "sum_n": int(sum(q.n for q in qps)),
                   "sum_m": int(sum(q.m for q in qps)), "tol": args.tol,
                   "precision": "fp32-products/fp64-reductions" if args.precision == 1 else "fp64"},
        "solve": {"solved": solved, "iters_mean": float(np.mean([r["iters"] for r in rs])),
                  "iters_max": int(max(r["iters"] for r in rs)),
                  "cg_steps_mean": float(np.mean([r["cg_iters_total"] for r in rs])),
                  "rel_kkt_max": float(max(r["rel_kkt"] for r in rs)), "create_s": create_s,
                  "kernel_s": kernel_s, "launches_per_solve": 1, "workgroup_threads": batch.threads,
                  "autotuner": tuned},
        "roofline": {"kernel": kernel_name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_alg},
    }
    if traffic is not None:
        line["roofline"]["traffic_over_algorithmic"] = traffic / bytes_alg
    batch.close()
    # the practical ceiling of the same GPU, measured after the timed region
    ceiling = stream_ceiling()
    line["roofline"]["stream_ceiling"] = ceiling
    if traffic is not None:
        line["roofline"]["measured_traffic_GBps"] = traffic / kernel_s / 1e9
    progress(f"device copy (read + write): {ceiling['copy_GBps']:.0f} GB/s")
    if not args.no_extras:
        extras = {}
        obo = one_by_one_sample(pairs, args)
        obo["speedup_of_batch_kernel_s"] = obo["estimated_kernel_s_all"] / kernel_s
        extras["one_by_one_single_qp"] = obo
        extras["random_qp_1e5"] = side_random1e5(args)
        progress(f"random QP n=1e5: {extras['random_qp_1e5']['kernel_ms']:.1f} ms per solve")
        extras["powerlaw_2e6"] = side_powerlaw(args)
        progress(f"power-law n=2e6: {extras['powerlaw_2e6']['status']} in {extras['powerlaw_2e6']['kernel_ms']:.1f} ms")
        extras["learned_warm_start"] = side_warm_start(args)
        line["extras"] = extras
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_portfolio(count, args.tol)
    print(json.dumps(line), flush=True)
    torch.cuda.synchronize()


def bench_random1e5(args):
    """The random sparse QP n = 1e5 as its own bench line (single-QP solve
    kernel, FP32 products, cold start, tol 1e-4)."""
    import torch
    from paper_2405_16160_amd import pdhcg
    qp = workload()
    settings = pdhcg.Settings(tol_rel_kkt=args.tol, precision=args.precision, num_blocks=args.num_blocks)
    solver = pdhcg.Solver(qp, settings)
    plan = solver.plan_info()
    for _ in range(args.warmup):
        x, y, r = solver.solve()
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, y, r = solver.solve()
        results.append(r)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert all(rr["status"] == 0 for rr in results), [rr["status_name"] for rr in results]
    r = results[-1]
    kernel_s = float(np.mean([rr["kernel_s"] for rr in results]))
    launches = 1   # one solve-kernel launch per solve at this size (5000-iteration chunks)
    bytes_alg = solve_bytes(qp, r, args.precision)
    achieved = bytes_alg / kernel_s / 1e9
    traffic, _ = measured_traffic(os.path.join(ROOT, "profiles", "pdhcg_solve_kernel_random_qp_1e5_counters.md"))
    line = {
        "metric": "time & QPs/s to rel. KKT<=1e-4 (batched/warm-start vs plain); SpMV HBM GB/s",
        "value": args.steps / dt,
        "unit": "QPs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == 1 else "f64",
        "data": "synthetic",
        "config": {"workload": "plain PDHCG, random sparse convex QP n=1e5 m=5e4 (R 5e4x1e5 at 2e-5, "
                               "A at 2e-4), FP32 products + FP64 reductions, cold start, tol 1e-4",
                   "n": qp.n, "m": qp.m, "nnz_Q": qp.Q.nnz, "nnz_A": qp.A.nnz, "tol": args.tol,
                   "precision": "fp32-products/fp64-reductions" if args.precision == 1 else "fp64",
                   "plan": plan},
        "solve": {"iters": r["iters"], "cg_steps": r["cg_iters_total"], "restarts": r["restarts"],
                  "kkt_evals": r["kkt_evals"], "rel_kkt": r["rel_kkt"], "setup_s": r["setup_s"],
                  "kernel_ms": kernel_s * 1e3, "launches_per_solve": launches},
        "roofline": {"kernel": "pdhcg_solve_kernel", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": bytes_alg / launches,
                     # the HBM roofline is the reference, not what limits this instance
                     "limited_by": "latency: a grid barrier and a few dependent round trips per phase; Q and A "
                                   "(about 16 MB) stay in the 256 MB MALL between phases"},
    }
    if traffic is not None:
        line["roofline"]["traffic_over_algorithmic"] = traffic / (bytes_alg / launches)
    if not args.no_extras:
        extras = spmv_rates(solver, qp, reps=200)
        # in-run comparison: CG capped at one step (linearised primal step)
        s1 = pdhcg.Settings(tol_rel_kkt=args.tol, precision=args.precision, num_blocks=args.num_blocks,
                            max_cg_iters=1, cg_rule=1, max_iters=200_000)
        solver.set_settings(s1)
        t = time.perf_counter()
        _, _, r1 = solver.solve()
        torch.cuda.synchronize()
        extras["cg_cap_1"] = {"seconds": time.perf_counter() - t, "iters": r1["iters"], "status": r1["status_name"],
                              "speedup_of_pdhcg": (time.perf_counter() - t) / (dt / args.steps)}
        solver.set_settings(settings)
        extras["spmv_cold"] = spmv_cold_rates(solver, qp)
        extras["instances_0_9"] = instances_geomean(args)
        line["extras"] = extras
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(qp, args.tol)
    print(json.dumps(line), flush=True)
    solver.close()
    torch.cuda.synchronize()




if __name__ == "__main__":
    main()
