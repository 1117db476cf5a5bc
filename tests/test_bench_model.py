"""The measurement code of bench.py (no GPU): the compulsory-byte model of a
product and of a solve, and the scaling of the HBM counters by the copy
calibration, on hand-made inputs."""
import csv
import os

import numpy as np

import bench
from paper_2405_16160_amd import instances as I


def test_csr_bytes_counts_matrix_vector_and_result_once():
    # 10 nonzeros of a 4 x 6 matrix, FP32 values and x, FP64 y:
    # values 40 + columns 40 + row pointers 20 + x 24 + y 32
    assert bench.csr_bytes(10, 4, 6, 4, 4, 8) == 40 + 40 + 20 + 24 + 32
    # FP64 throughout: values 80 + columns 40 + row pointers 20 + x 48 + y 32
    assert bench.csr_bytes(10, 4, 6, 8, 8) == 80 + 40 + 20 + 48 + 32


def test_solve_bytes_grow_with_the_reported_counts():
    qp = I.random_qp(family=1, instance=0)
    base = {"iters": 10, "cg_iters_total": 30, "kkt_evals": 1}
    b0 = bench.solve_bytes(qp, base, 1)
    more_cg = bench.solve_bytes(qp, dict(base, cg_iters_total=31), 1)
    # one more CG step adds nnz(Q)(4 + 4) + 4(n + 1) + 11 n 4 bytes in FP32 products
    n = qp.n
    assert more_cg - b0 == qp.Q.nnz * 8 + 4 * (n + 1) + 11 * n * 4
    # FP64 products move more bytes than FP32 ones
    assert bench.solve_bytes(qp, base, 0) > b0


def test_factored_q_counts_the_factor_not_the_dense_matrix():
    qp = I.portfolio_qp(3, nmax=300)
    r = {"iters": 5, "cg_iters_total": 20, "kkt_evals": 0}
    k = -(-qp.n // 10)
    dense = bench.solve_bytes(qp, r, 1, dense_q=True)
    fact = bench.solve_bytes(qp, r, 1, dense_q=True, rank=k)
    # per CG step the dense form streams n^2 FP32 values, the factored form 2nk + n
    one_more = dict(r, cg_iters_total=21)
    assert bench.solve_bytes(qp, one_more, 1, dense_q=True) - dense - (
        bench.solve_bytes(qp, one_more, 1, dense_q=True, rank=k) - fact) == (qp.n * qp.n - (2 * qp.n * k + qp.n)) * 4


def _write_csv(path, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_counter_summary_scales_by_the_copy_calibration(tmp_path):
    d = str(tmp_path)
    gib_kib = bench.CALIBRATION_BYTES / 1024.0
    # the copy reads 1 GiB (counter shows half: factor 0.5) and writes 1 GiB (factor 1)
    _write_csv(os.path.join(d, "copy_fetch", "run_counter_collection.csv"),
               [{"Kernel_Name": "copyBuffer", "Counter_Name": "FETCH_SIZE", "Counter_Value": gib_kib / 2}])
    _write_csv(os.path.join(d, "copy_write", "run_counter_collection.csv"),
               [{"Kernel_Name": "copyBuffer", "Counter_Name": "WRITE_SIZE", "Counter_Value": gib_kib}])
    _write_csv(os.path.join(d, "fetch", "run_counter_collection.csv"),
               [{"Kernel_Name": "pdhcg::pdhcg_solve_kernel(x)", "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000.0},
                {"Kernel_Name": "other", "Counter_Name": "FETCH_SIZE", "Counter_Value": 5.0}])
    _write_csv(os.path.join(d, "write", "run_counter_collection.csv"),
               [{"Kernel_Name": "pdhcg::pdhcg_solve_kernel(x)", "Counter_Name": "WRITE_SIZE", "Counter_Value": 300.0}])
    s = bench.summarize_counters(d, 1e6, kernel="pdhcg_solve_kernel")
    assert np.isclose(s["counters"]["FETCH_SIZE"]["factor"], 0.5)
    assert np.isclose(s["counters"]["FETCH_SIZE"]["bytes_per_launch"], 1000.0 * 1024 / 0.5)
    assert np.isclose(s["counters"]["WRITE_SIZE"]["bytes_per_launch"], 300.0 * 1024)
    assert np.isclose(s["traffic_bytes_per_launch"], 1000.0 * 1024 / 0.5 + 300.0 * 1024)
    assert np.isclose(s["traffic_over_algorithmic"], s["traffic_bytes_per_launch"] / 1e6)
