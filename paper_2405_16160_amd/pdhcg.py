"""Python binding of the C ABI in ``include/pdhcg.h`` (argument marshalling only).

Every step of the solver runs in the HIP library ``libpdhcg.so``; this module
only converts arrays and settings.  Device-resident data are torch tensors on
the current HIP device and are handed over by pointer together with torch's
current stream.  There is no CPU fallback: if the library cannot be loaded,
``lib()`` raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import dataclasses
import os
import weakref

import numpy as np

from . import build as _build

_lib = None
_live = weakref.WeakSet()   # open Solver / mlp.Network objects, closed at interpreter exit


@atexit.register
def _close_live():
    """Release every handle still open while the HIP runtime and torch are
    fully alive (Python's exit handlers run before its module teardown and
    before the C runtime's), after the device has finished its work."""
    objs = list(_live)
    if not objs:
        return
    try:
        import torch
        torch.cuda.synchronize()
    except Exception:
        pass
    for o in objs:
        try:
            o.close()
        except Exception:
            pass


class pdhcg_csr(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64), ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("on_device", C.c_int32)]


class pdhcg_settings(C.Structure):
    _fields_ = [("tol_rel_kkt", C.c_double), ("max_iters", C.c_int64), ("max_cg_iters", C.c_int32),
                ("cg_rule", C.c_int32), ("cg_eps_factor", C.c_double), ("beta_sufficient", C.c_double),
                ("beta_necessary", C.c_double), ("beta_artificial", C.c_double), ("restart_to", C.c_int32),
                ("eval_period", C.c_int32), ("primal_weight_theta", C.c_double),
                ("primal_weight_init", C.c_double), ("step_eta_factor", C.c_double), ("power_iters", C.c_int32),
                ("precision", C.c_int32), ("time_limit_s", C.c_double), ("num_blocks", C.c_int32),
                ("warm_fallback", C.c_int32), ("verbose", C.c_int32), ("cg_form", C.c_int32),
                ("ruiz_iters", C.c_int32), ("pock_chambolle", C.c_int32), ("step_rule", C.c_int32),
                ("threads", C.c_int32)]


class pdhcg_lowrank(C.Structure):
    _fields_ = [("n", C.c_int64), ("k", C.c_int64), ("F", C.c_void_p), ("d", C.c_void_p), ("on_device", C.c_int32)]


class pdhcg_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("returned_average", C.c_int32), ("rel_primal", C.c_double),
                ("rel_dual", C.c_double), ("rel_gap", C.c_double), ("rel_kkt", C.c_double),
                ("primal_obj", C.c_double), ("dual_obj", C.c_double), ("iters", C.c_int64),
                ("cg_iters_total", C.c_int64), ("restarts", C.c_int64), ("norm_A", C.c_double),
                ("setup_s", C.c_double), ("solve_s", C.c_double), ("kernel_s", C.c_double),
                ("kkt_evals", C.c_int64), ("cold_fallback", C.c_int32), ("rejected_steps", C.c_int64),
                ("step_eta", C.c_double), ("qx_formed", C.c_int64)]


STATUS = {0: "OPTIMAL", 1: "ITERATION_LIMIT", 2: "TIME_LIMIT", 3: "NUMERICAL_ERROR"}
EXPORTS = ["pdhcg_default_settings", "pdhcg_create", "pdhcg_create_lowrank", "pdhcg_set_settings", "pdhcg_set_b",
           "pdhcg_solve", "pdhcg_solve_batch", "pdhcg_solve_batch_noalloc", "pdhcg_solve_batch_lowrank",
           "pdhcg_solve_multi_rhs", "pdhcg_spmv", "pdhcg_get_scaling",
           "pdhcg_autotune", "pdhcg_plan_info", "pdhcg_destroy", "pdhcg_error_string", "pdhcg_last_error",
           "pdhcg_batch_create", "pdhcg_batch_layout", "pdhcg_batch_solve", "pdhcg_batch_get_scaling",
           "pdhcg_batch_set_threads", "pdhcg_batch_autotune", "pdhcg_batch_destroy"]


class PdhcgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pdhcg error {code}: {msg}")
        self.code = code


def lib_path() -> str:
    return _build.LIB


def lib():
    """Load libpdhcg.so (building it first only when it does not exist)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        # torch ships its own HIP runtime under a different file name; loading
        # torch first makes the library bind to that same runtime (loading the
        # library first would put a second HIP runtime in the process, and the
        # two then fail each other's allocations)
        import torch  # noqa: F401
        L = C.CDLL(_build.LIB)
        P = C.c_void_p
        L.pdhcg_default_settings.argtypes = [C.POINTER(pdhcg_settings)]
        L.pdhcg_default_settings.restype = None
        L.pdhcg_create.argtypes = [C.POINTER(P), C.POINTER(pdhcg_csr), C.POINTER(pdhcg_csr), P, P, C.c_int32,
                                   C.POINTER(pdhcg_settings), P]
        L.pdhcg_create_lowrank.argtypes = [C.POINTER(P), C.POINTER(pdhcg_csr), P, C.POINTER(pdhcg_csr), P, P,
                                           C.c_int32, C.POINTER(pdhcg_settings), P]
        L.pdhcg_set_settings.argtypes = [P, C.POINTER(pdhcg_settings)]
        L.pdhcg_set_b.argtypes = [P, P, C.c_int32]
        L.pdhcg_solve.argtypes = [P, P, P, P, P, C.c_int32, C.POINTER(pdhcg_result)]
        L.pdhcg_solve_batch.argtypes = [C.c_int32, P, P, P, P, P, P, P, P, P, C.POINTER(pdhcg_settings), P]
        L.pdhcg_solve_batch_noalloc.argtypes = [C.c_int32, P, P, P, P, P, P, P, P, P, C.POINTER(pdhcg_settings), P]
        L.pdhcg_solve_batch_lowrank.argtypes = [C.c_int32, P, P, P, P, P, P, P, P, P, C.POINTER(pdhcg_settings), P]
        L.pdhcg_solve_multi_rhs.argtypes = [C.c_int32, C.POINTER(pdhcg_csr), C.POINTER(pdhcg_csr), P, P, P, P, P, P,
                                            P, C.POINTER(pdhcg_settings), P]
        L.pdhcg_spmv.argtypes = [P, C.c_int32, C.c_int32, P, P, C.c_int32]
        L.pdhcg_plan_info.argtypes = [P, P, P, P, P, P, P]
        L.pdhcg_get_scaling.argtypes = [P, P, P, C.c_int32]
        L.pdhcg_autotune.argtypes = [P, C.c_int32, P, P]
        L.pdhcg_destroy.argtypes = [P]
        L.pdhcg_destroy.restype = None
        L.pdhcg_error_string.argtypes = [C.c_int]
        L.pdhcg_error_string.restype = C.c_char_p
        L.pdhcg_last_error.argtypes = []
        L.pdhcg_last_error.restype = C.c_char_p
        L.pdhcg_batch_create.argtypes = [C.POINTER(P), C.c_int32, P, P, P, P, P, C.c_int32, C.POINTER(pdhcg_settings), P]
        L.pdhcg_batch_layout.argtypes = [P, P, P]
        L.pdhcg_batch_solve.argtypes = [P, P, P, P, P, C.c_int32, P]
        L.pdhcg_batch_get_scaling.argtypes = [P, P, P, C.c_int32]
        L.pdhcg_batch_set_threads.argtypes = [P, C.c_int32]
        L.pdhcg_batch_autotune.argtypes = [P, C.c_int32, P, P]
        L.pdhcg_batch_destroy.argtypes = [P]
        L.pdhcg_batch_destroy.restype = None
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise PdhcgError(rc, lib().pdhcg_last_error().decode())


@dataclasses.dataclass
class Settings:
    """Mirror of pdhcg_settings (defaults as pdhcg_default_settings)."""
    tol_rel_kkt: float = 1e-4
    max_iters: int = 100000
    max_cg_iters: int = 100
    cg_rule: int = 0
    cg_eps_factor: float = 0.05
    beta_sufficient: float = 0.2
    beta_necessary: float = 0.8
    beta_artificial: float = 0.2
    restart_to: int = 0
    eval_period: int = 64
    primal_weight_theta: float = 0.2
    primal_weight_init: float = 1.0
    step_eta_factor: float = 0.5
    power_iters: int = 100
    precision: int = 0
    time_limit_s: float = 0.0
    num_blocks: int = 0
    warm_fallback: int = 1
    verbose: int = 0
    cg_form: int = 0
    ruiz_iters: int = 0
    pock_chambolle: int = 0
    step_rule: int = 0
    threads: int = 0

    def c(self) -> pdhcg_settings:
        s = pdhcg_settings()
        for f in dataclasses.fields(self):
            setattr(s, f.name, getattr(self, f.name))
        return s


def default_settings() -> Settings:
    s = pdhcg_settings()
    lib().pdhcg_default_settings(C.byref(s))
    return Settings(**{f.name: getattr(s, f.name) for f in dataclasses.fields(Settings)})


def _result_dict(r: pdhcg_result) -> dict:
    d = {name: getattr(r, name) for name, _ in pdhcg_result._fields_}
    d["status_name"] = STATUS.get(r.status, str(r.status))
    return d


def _stream_ptr():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Solver:
    """One QP on the GPU: ``Solver(qp, settings)`` then ``solve()``.

    ``qp`` is an ``instances.QP`` (host CSR, FP64).  The matrices and vectors
    are first moved to torch device tensors and handed to pdhcg_create as
    device pointers.  With ``lowrank=(P, d)`` (P an instances.CSR n x k, d an
    n-vector or None) Q = P P' + diag(d) is given in low-rank form through
    pdhcg_create_lowrank, and ``qp.Q`` is not read."""

    def __init__(self, qp, settings: Settings | None = None, lowrank=None):
        import torch
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.n, self.m = qp.A.ncols, qp.A.nrows
        self.settings = settings or Settings()
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt).to(self.dev)
        keep = []

        def csr(M):
            rp, col, val = t(M.rowptr, torch.int64), t(M.col, torch.int32), t(M.val, torch.float64)
            keep.extend([rp, col, val])
            return pdhcg_csr(M.nrows, M.ncols, int(M.rowptr[-1]), rp.data_ptr(), col.data_ptr() if col.numel() else None,
                             val.data_ptr() if val.numel() else None, 1)

        Ac = csr(qp.A)
        b = t(qp.b, torch.float64) if self.m else torch.zeros(1, dtype=torch.float64, device=self.dev)
        c = t(qp.c, torch.float64)
        h = C.c_void_p()
        if lowrank is not None:
            Pc = csr(lowrank[0])
            d = None if lowrank[1] is None else t(lowrank[1], torch.float64)
            torch.cuda.synchronize()
            _check(lib().pdhcg_create_lowrank(C.byref(h), C.byref(Pc), None if d is None else d.data_ptr(),
                                              C.byref(Ac), b.data_ptr(), c.data_ptr(), 1,
                                              C.byref(self.settings.c()), _stream_ptr()))
        else:
            Qc = csr(qp.Q)
            torch.cuda.synchronize()
            _check(lib().pdhcg_create(C.byref(h), C.byref(Qc), C.byref(Ac), b.data_ptr(), c.data_ptr(), 1,
                                      C.byref(self.settings.c()), _stream_ptr()))
        self.h = h
        _live.add(self)
        del keep

    def set_settings(self, settings: Settings):
        self.settings = settings
        _check(lib().pdhcg_set_settings(self.h, C.byref(settings.c())))

    def set_b(self, b):
        import torch
        bt = torch.as_tensor(np.ascontiguousarray(b), dtype=torch.float64).to(self.dev)
        _check(lib().pdhcg_set_b(self.h, bt.data_ptr(), 1))

    def solve(self, x0=None, y0=None, out=None):
        """Returns (x, y, result) with x, y as float64 device tensors."""
        import torch
        if out is None:
            x = torch.empty(self.n, dtype=torch.float64, device=self.dev)
            y = torch.empty(max(self.m, 1), dtype=torch.float64, device=self.dev)
        else:
            x, y = out
        dv = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float64).to(self.dev).contiguous()
        x0t, y0t = dv(x0), dv(y0)
        r = pdhcg_result()
        _check(lib().pdhcg_solve(self.h, None if x0t is None else x0t.data_ptr(),
                                 None if y0t is None else y0t.data_ptr(), x.data_ptr(), y.data_ptr(), 1, C.byref(r)))
        return x, y[: self.m], _result_dict(r)

    def spmv(self, which: int, x, precision: int = 0, repeats: int = 1, out=None):
        import torch
        nrows = self.n if which in (0, 2) else self.m
        xt = torch.as_tensor(x, dtype=torch.float64).to(self.dev).contiguous()
        y = out if out is not None else torch.empty(max(nrows, 1), dtype=torch.float64, device=self.dev)
        _check(lib().pdhcg_spmv(self.h, which, precision, xt.data_ptr(), y.data_ptr(), repeats))
        return y[:nrows]

    def scaling(self):
        """(d1, d2): the diagonals D1 (m) and D2 (n) of the preconditioning, as
        float64 device tensors (ones when it is off)."""
        import torch
        d1 = torch.empty(max(self.m, 1), dtype=torch.float64, device=self.dev)
        d2 = torch.empty(self.n, dtype=torch.float64, device=self.dev)
        _check(lib().pdhcg_get_scaling(self.h, d1.data_ptr(), d2.data_ptr(), 1))
        return d1[: self.m], d2

    def autotune(self, iters: int = 50) -> dict:
        nb, g = C.c_int32(), C.c_int32()
        _check(lib().pdhcg_autotune(self.h, iters, C.byref(nb), C.byref(g)))
        threads = self.plan_info()["threads"]
        self.settings.num_blocks = nb.value
        self.settings.threads = threads
        return {"num_blocks": nb.value, "group_scale": g.value, "threads": threads}

    def plan_info(self) -> dict:
        v = [C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64(), C.c_int32()]
        _check(lib().pdhcg_plan_info(self.h, *[C.byref(a) for a in v]))
        return dict(num_blocks=v[0].value, group_n=v[1].value, group_q=v[2].value, group_m=v[3].value,
                    long_rows=v[4].value, threads=v[5].value)

    def close(self):
        if getattr(self, "h", None):
            lib().pdhcg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(qps, settings: Settings | None = None, x0s=None, y0s=None, lowrank=None, noalloc=False):
    """Solve a list of QPs with pdhcg_solve_batch (host arrays in and out).
    lowrank: optional list of (F, d) with Q_i = F F' + diag(d) (then
    pdhcg_solve_batch_lowrank; qps[i].Q is not read).  noalloc: use
    pdhcg_solve_batch_noalloc (device buffers carved from the library's static
    scratch; CSR Q only).  Returns a list of (x, y, result) with numpy
    arrays."""
    settings = settings or Settings()
    cnt = len(qps)
    keep = []
    Qs = (pdhcg_csr * cnt)()
    Ls = (pdhcg_lowrank * cnt)() if lowrank is not None else None
    As = (pdhcg_csr * cnt)()
    bs = (C.c_void_p * cnt)()
    cs = (C.c_void_p * cnt)()
    xo = (C.c_void_p * cnt)()
    yo = (C.c_void_p * cnt)()
    x0 = (C.c_void_p * cnt)() if x0s is not None else None
    y0 = (C.c_void_p * cnt)() if y0s is not None else None
    outs = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a

    for i, qp in enumerate(qps):
        if Ls is not None:
            F, d = arr(lowrank[i][0], np.float64), arr(lowrank[i][1], np.float64)
            Ls[i] = pdhcg_lowrank(F.shape[0], F.shape[1], F.ctypes.data, d.ctypes.data, 0)
        for M, dst in (((qp.A, As),) if Ls is not None else ((qp.Q, Qs), (qp.A, As))):
            rp, col, val = arr(M.rowptr, np.int64), arr(M.col, np.int32), arr(M.val, np.float64)
            dst[i] = pdhcg_csr(M.nrows, M.ncols, int(M.rowptr[-1]), rp.ctypes.data, col.ctypes.data,
                               val.ctypes.data, 0)
        bs[i] = arr(qp.b if qp.A.nrows else np.zeros(1), np.float64).ctypes.data
        cs[i] = arr(qp.c, np.float64).ctypes.data
        xv = np.zeros(qp.Q.nrows)
        yv = np.zeros(max(qp.A.nrows, 1))
        outs.append((xv, yv))
        xo[i] = xv.ctypes.data
        yo[i] = yv.ctypes.data
        if x0 is not None and x0s[i] is not None:
            x0[i] = arr(x0s[i], np.float64).ctypes.data
        if y0 is not None and y0s[i] is not None:
            y0[i] = arr(y0s[i], np.float64).ctypes.data
    rs = (pdhcg_result * cnt)()
    if Ls is not None:
        if noalloc:
            raise ValueError("the allocation-free entry point takes Q in CSR form only")
        _check(lib().pdhcg_solve_batch_lowrank(cnt, Ls, As, bs, cs, x0, y0, xo, yo, rs, C.byref(settings.c()),
                                               _stream_ptr()))
    else:
        fn = lib().pdhcg_solve_batch_noalloc if noalloc else lib().pdhcg_solve_batch
        _check(fn(cnt, Qs, As, bs, cs, x0, y0, xo, yo, rs, C.byref(settings.c()), _stream_ptr()))
    return [(outs[i][0], outs[i][1][: qps[i].A.nrows], _result_dict(rs[i])) for i in range(cnt)]


def solve_multi_rhs(Q, A, c, B, settings: Settings | None = None, X0=None, Y0=None):
    """Solve the QPs (Q, A, B[i], c) for the rows B[i] of B (count x m) with
    pdhcg_solve_multi_rhs (host arrays).  X0 / Y0: count x n / count x m start
    points or None.  Returns (X, Y, results) with X count x n, Y count x m."""
    settings = settings or Settings()
    B = np.ascontiguousarray(B, dtype=np.float64)
    cnt, n, m = B.shape[0], Q.nrows, A.nrows
    keep = []

    def csr(M):
        rp, col, val = (np.ascontiguousarray(M.rowptr, np.int64), np.ascontiguousarray(M.col, np.int32),
                        np.ascontiguousarray(M.val, np.float64))
        keep.extend((rp, col, val))
        return pdhcg_csr(M.nrows, M.ncols, int(M.rowptr[-1]), rp.ctypes.data, col.ctypes.data, val.ctypes.data, 0)

    def opt(a, shape):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64).reshape(shape)
        keep.append(a)
        return a.ctypes.data

    cv = np.ascontiguousarray(c, dtype=np.float64)
    X = np.zeros((cnt, n))
    Y = np.zeros((cnt, max(m, 1)))
    rs = (pdhcg_result * cnt)()
    Qc, Ac = csr(Q), csr(A)
    _check(lib().pdhcg_solve_multi_rhs(cnt, C.byref(Qc), C.byref(Ac), B.ctypes.data, cv.ctypes.data,
                                       opt(X0, (cnt, n)), opt(Y0, (cnt, m)), X.ctypes.data, Y.ctypes.data, rs,
                                       C.byref(settings.c()), _stream_ptr()))
    return X, Y[:, :m], [_result_dict(rs[i]) for i in range(cnt)]


class Batch:
    """A batch packed on the device once (pdhcg_batch_create) and solved any
    number of times (pdhcg_batch_solve) with device-resident start points and
    outputs: ``Batch(qps, settings, lowrank=None)`` then ``solve()``.

    ``qps`` are ``instances.QP`` objects (host CSR); with ``lowrank`` (a list
    of (F, d) with Q_i = F F' + diag(d)) their Q is not read.  Matrices and
    vectors are handed over as host arrays (the library copies them once)."""

    def __init__(self, qps, settings: Settings | None = None, lowrank=None, device_inputs: bool = False):
        import torch
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self.settings = settings or Settings()
        self.count = cnt = len(qps)
        self.threads = 256
        keep = []
        on_dev = 1 if device_inputs else 0
        tdt = {np.int64: torch.int64, np.int32: torch.int32, np.float64: torch.float64}

        class _Ptr:  # what a ctypes field needs from a host array or a device tensor
            def __init__(self, data):
                self.data = data

        def arr(a, dt):
            """a host array, or (device_inputs) a device tensor; .ctypes.data is its address"""
            a = np.ascontiguousarray(a, dtype=dt)
            if device_inputs:
                t = torch.as_tensor(a, dtype=tdt[dt]).to(self.dev)
                keep.append(t)
                return type("DevArr", (), {"ctypes": _Ptr(t.data_ptr() if t.numel() else None), "shape": a.shape})()
            keep.append(a)
            return a

        Qs = (pdhcg_csr * cnt)() if lowrank is None else None
        Ls = (pdhcg_lowrank * cnt)() if lowrank is not None else None
        As = (pdhcg_csr * cnt)()
        bs = (C.c_void_p * cnt)()
        cs = (C.c_void_p * cnt)()
        for i, qp in enumerate(qps):
            if Ls is not None:
                F, d = arr(lowrank[i][0], np.float64), arr(lowrank[i][1], np.float64)
                Ls[i] = pdhcg_lowrank(F.shape[0], F.shape[1], F.ctypes.data, d.ctypes.data, on_dev)
            for M, dst in (((qp.A, As),) if Ls is not None else ((qp.Q, Qs), (qp.A, As))):
                rp, col, val = arr(M.rowptr, np.int64), arr(M.col, np.int32), arr(M.val, np.float64)
                dst[i] = pdhcg_csr(M.nrows, M.ncols, int(M.rowptr[-1]), rp.ctypes.data, col.ctypes.data,
                                   val.ctypes.data, on_dev)
            bs[i] = arr(qp.b if qp.A.nrows else np.zeros(1), np.float64).ctypes.data
            cs[i] = arr(qp.c, np.float64).ctypes.data
        h = C.c_void_p()
        if device_inputs:
            torch.cuda.synchronize()
        _check(lib().pdhcg_batch_create(C.byref(h), cnt, Qs, Ls, As, bs, cs, on_dev, C.byref(self.settings.c()),
                                        _stream_ptr()))
        self.h = h
        _live.add(self)
        del keep
        n_off = np.zeros(cnt + 1, dtype=np.int64)
        m_off = np.zeros(cnt + 1, dtype=np.int64)
        _check(lib().pdhcg_batch_layout(self.h, n_off.ctypes.data, m_off.ctypes.data))
        self.n_off, self.m_off = n_off, m_off
        self.x = torch.empty(int(n_off[-1]), dtype=torch.float64, device=self.dev)
        self.y = torch.empty(max(int(m_off[-1]), 1), dtype=torch.float64, device=self.dev)

    def solve(self, x0=None, y0=None):
        """Solve all instances; x0 / y0: packed float64 device tensors or None.
        Returns (x, y, results) with x, y the packed device outputs (views
        that the next solve overwrites) and one result dict per instance."""
        rs = (pdhcg_result * self.count)()
        ptr = lambda t: None if t is None else t.contiguous().data_ptr()
        _check(lib().pdhcg_batch_solve(self.h, ptr(x0), ptr(y0), self.x.data_ptr(), self.y.data_ptr(), 1, rs))
        return self.x, self.y[: int(self.m_off[-1])], [_result_dict(rs[i]) for i in range(self.count)]

    def set_threads(self, threads: int):
        """Threads per workgroup of the batched kernel: 256 (default) or 512."""
        _check(lib().pdhcg_batch_set_threads(self.h, threads))
        self.threads = threads

    def autotune(self, reps: int = 1) -> dict:
        """Time cold solves of the whole batch at 256 and 512 threads per
        workgroup and keep the faster; returns the choice and both times."""
        t = C.c_int32()
        ks = (C.c_double * 2)()
        _check(lib().pdhcg_batch_autotune(self.h, reps, C.byref(t), ks))
        self.threads = t.value
        return {"threads": t.value, "kernel_s": {256: ks[0], 512: ks[1]}}

    def split(self, x, y):
        """Per-instance numpy views of packed x, y."""
        xs, ys = x.cpu().numpy(), y.cpu().numpy()
        return ([xs[self.n_off[i]:self.n_off[i + 1]] for i in range(self.count)],
                [ys[self.m_off[i]:self.m_off[i + 1]] for i in range(self.count)])

    def scaling(self):
        """(d1, d2) packed (ones when preconditioning is off), device tensors."""
        import torch
        d1 = torch.empty(max(int(self.m_off[-1]), 1), dtype=torch.float64, device=self.dev)
        d2 = torch.empty(int(self.n_off[-1]), dtype=torch.float64, device=self.dev)
        _check(lib().pdhcg_batch_get_scaling(self.h, d1.data_ptr(), d2.data_ptr(), 1))
        return d1[: int(self.m_off[-1])], d2

    def close(self):
        if getattr(self, "h", None):
            lib().pdhcg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
