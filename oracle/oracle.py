"""ctypes front end of the FP64 CPU oracle (``pdhcg_oracle.c``).

TEST INFRASTRUCTURE ONLY: this module exists so that the test suite, the smoke
check and the CPU-baseline leg of the benchmark can run the reference
implementation.  The GPU library never imports it, and it imports nothing from
the GPU library.  ``build()`` compiles the C source with gcc (OpenMP on the
row loops of the sparse products).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdhcg_oracle.c")
_LIB = os.path.join(_HERE, "libpdhcg_oracle.so")

OPTIMAL, ITER_LIMIT, NUMERICAL_ERROR = 0, 1, 3


class _Csr(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64), ("rowptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p)]


class _Original(C.Structure):
    _fields_ = [("Q", C.POINTER(_Csr)), ("A", C.POINTER(_Csr)), ("b", C.c_void_p), ("c", C.c_void_p),
                ("d1", C.c_void_p), ("d2", C.c_void_p)]


class _Settings(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iters", C.c_int64), ("max_cg", C.c_int32),
                ("cg_rule", C.c_int32), ("cg_eps_factor", C.c_double), ("beta_suf", C.c_double),
                ("beta_nec", C.c_double), ("beta_art", C.c_double), ("restart_to", C.c_int32),
                ("eval_period", C.c_int32), ("pw_theta", C.c_double), ("pw_init", C.c_double),
                ("eta_factor", C.c_double), ("power_iters", C.c_int32), ("step_rule", C.c_int32)]


@dataclass
class Settings:
    """Oracle settings; defaults are the paper's constants and the readings
    documented in ``pdhcg_oracle.c``."""
    tol: float = 1e-6
    max_iters: int = 100_000
    max_cg: int = 100
    cg_rule: int = 0
    cg_eps_factor: float = 0.05
    beta_suf: float = 0.2
    beta_nec: float = 0.8
    beta_art: float = 0.2
    restart_to: int = 0
    eval_period: int = 64
    pw_theta: float = 0.2
    pw_init: float = 1.0
    eta_factor: float = 0.5
    power_iters: int = 100
    step_rule: int = 0   # 0: constant eta per epoch, 1: adaptive step (Sec. 4)

    def _c(self) -> _Settings:
        return _Settings(self.tol, self.max_iters, self.max_cg, self.cg_rule, self.cg_eps_factor,
                         self.beta_suf, self.beta_nec, self.beta_art, self.restart_to, self.eval_period,
                         self.pw_theta, self.pw_init, self.eta_factor, self.power_iters, self.step_rule)


@dataclass
class Result:
    x: np.ndarray
    y: np.ndarray
    status: int
    iters: int
    cg_steps: int
    restarts: int
    returned_average: bool
    r_primal: float
    r_dual: float
    r_gap: float
    rel_kkt: float
    primal_obj: float
    dual_obj: float
    norm_A: float
    rejections: int = 0
    trace_x: np.ndarray | None = None
    trace_y: np.ndarray | None = None
    trace_xa: np.ndarray | None = None
    trace_ya: np.ndarray | None = None
    trace_cg: np.ndarray | None = None
    trace_step: np.ndarray | None = None   # per iteration: eta used, its limit eta_bar, attempts


def build(force: bool = False) -> str:
    """Compile the oracle into ``libpdhcg_oracle.so`` next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lib_path = None


def use_library(path=None):
    """Load the oracle from another compiled copy of pdhcg_oracle.c (the
    mutation tests build copies with a planted mistake); None restores the
    default library."""
    global _lib, _lib_path
    _lib, _lib_path = None, path


def lib():
    global _lib
    if _lib is None:
        if _lib_path is None:
            build()
        L = C.CDLL(_lib_path or _LIB)
        P = C.c_void_p
        L.or_matvec.argtypes = [C.POINTER(_Csr), P, P]
        L.or_matvec_t.argtypes = [C.POINTER(_Csr), P, P]
        L.or_kkt.argtypes = [C.POINTER(_Csr), C.POINTER(_Csr), P, P, P, P, P]
        L.or_opnorm.argtypes = [C.POINTER(_Csr), C.c_int32]
        L.or_opnorm.restype = C.c_double
        L.or_cg.argtypes = [C.POINTER(_Csr), C.c_double, P, P, C.c_double, C.c_int32, C.c_int32]
        L.or_cg.restype = C.c_int32
        L.or_restart_decision.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int64, C.c_int64,
                                          C.c_double, C.c_double, C.c_double]
        L.or_restart_decision.restype = C.c_int32
        L.or_primal_weight.argtypes = [C.c_double] * 4
        L.or_primal_weight.restype = C.c_double
        L.or_solve.argtypes = [C.POINTER(_Csr), C.POINTER(_Csr), P, P, C.POINTER(_Settings), P, P, P, P, P,
                               C.c_int64, P, P, P, P, P, P, C.POINTER(_Original)]
        L.or_step_limit.argtypes = [C.POINTER(_Csr), C.POINTER(_Csr), P, P, P, P, C.c_double]
        L.or_step_limit.restype = C.c_double
        L.or_next_step.argtypes = [C.c_double, C.c_double, C.c_int64]
        L.or_next_step.restype = C.c_double
        L.or_solve.restype = C.c_int32
        L.or_num_threads.restype = C.c_int32
        _lib = L
    return _lib


class _Mat:
    """Keeps contiguous copies alive while a C call uses them."""

    def __init__(self, M):
        self.rowptr = np.ascontiguousarray(M.rowptr, dtype=np.int64)
        self.col = np.ascontiguousarray(M.col, dtype=np.int32)
        self.val = np.ascontiguousarray(M.val, dtype=np.float64)
        self.c = _Csr(M.nrows, M.ncols, self.rowptr.ctypes.data, self.col.ctypes.data, self.val.ctypes.data)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return None if a is None else a.ctypes.data


def matvec(M, x):
    Mm = _Mat(M)
    x = _f64(x)
    y = np.zeros(M.nrows)
    lib().or_matvec(C.byref(Mm.c), _p(x), _p(y))
    return y


def matvec_t(M, y):
    Mm = _Mat(M)
    y = _f64(y)
    x = np.zeros(M.ncols)
    lib().or_matvec_t(C.byref(Mm.c), _p(y), _p(x))
    return x


def kkt(qp, x, y):
    """relKKT pieces: dict with r_primal, r_dual, r_gap, rel_kkt, primal_obj,
    dual_obj, xQx, by."""
    Q, A = _Mat(qp.Q), _Mat(qp.A)
    b, c, x, y = _f64(qp.b), _f64(qp.c), _f64(x), _f64(y)
    out = np.zeros(8)
    lib().or_kkt(C.byref(Q.c), C.byref(A.c), _p(b), _p(c), _p(x), _p(y), _p(out))
    keys = ["r_primal", "r_dual", "r_gap", "rel_kkt", "primal_obj", "dual_obj", "xQx", "by"]
    return dict(zip(keys, out.tolist()))


def opnorm(A, iters=100):
    Am = _Mat(A)
    return lib().or_opnorm(C.byref(Am.c), iters)


def cg(Q, tau, g, x, eps, max_steps, cg_rule=0):
    """One inexact CG solve; returns (x_new, steps)."""
    Qm = _Mat(Q)
    g = _f64(g)
    xn = _f64(x).copy()
    steps = lib().or_cg(C.byref(Qm.c), tau, _p(g), _p(xn), eps, max_steps, cg_rule)
    return xn, steps


def restart_decision(K_c, K_anchor, K_prev, k, k_total, beta_suf=0.2, beta_nec=0.8, beta_art=0.2):
    return lib().or_restart_decision(K_c, K_anchor, K_prev, k, k_total, beta_suf, beta_nec, beta_art)


def primal_weight(omega, dx, dy, theta=0.2):
    return lib().or_primal_weight(omega, dx, dy, theta)


def step_limit(qp, x, xn, y, yn, omega=1.0):
    """eta_bar of the adaptive step for the trial z = (x, y) -> (xn, yn)."""
    Q, A = _Mat(qp.Q), _Mat(qp.A)
    x, xn, y, yn = _f64(x), _f64(xn), _f64(y), _f64(yn)
    return lib().or_step_limit(C.byref(Q.c), C.byref(A.c), _p(x), _p(xn), _p(y), _p(yn), omega)


def next_step(eta, eta_bar, t):
    return lib().or_next_step(eta, eta_bar, t)


def num_threads():
    return lib().or_num_threads()


def solve(qp, settings: Settings | None = None, x0=None, y0=None, trace_len=0, original=None) -> Result:
    """Run the oracle on qp.  original = (qp0, d1, d2) declares qp a
    preconditioned copy of qp0 (Q = D2 Q0 D2, A = D1 A0 D2, b = D1 b0,
    c = D2 c0): every relKKT is then taken on qp0 at (D2 x, D1 y), and the
    reported residuals and objectives are qp0's; x, y stay those of qp."""
    s = settings or Settings()
    orig = None
    if original is not None:
        q0, d1, d2 = original
        Q0, A0 = _Mat(q0.Q), _Mat(q0.A)
        b0, c0, d1, d2 = _f64(q0.b), _f64(q0.c), _f64(d1), _f64(d2)
        orig_keep = (Q0, A0, b0, c0, d1, d2)  # noqa: F841 (alive during the call)
        orig = _Original(C.pointer(Q0.c), C.pointer(A0.c), _p(b0), _p(c0), _p(d1), _p(d2))
    Q, A = _Mat(qp.Q), _Mat(qp.A)
    n, m = qp.Q.nrows, qp.A.nrows
    b, c = _f64(qp.b), _f64(qp.c)
    x0 = None if x0 is None else _f64(x0)
    y0 = None if y0 is None else _f64(y0)
    x = np.zeros(n)
    y = np.zeros(m)
    info = np.zeros(13)
    tx = np.zeros(max(trace_len, 1) * n)
    ty = np.zeros(max(trace_len, 1) * m)
    txa = np.zeros(max(trace_len, 1) * n)
    tya = np.zeros(max(trace_len, 1) * m)
    tc = np.zeros(max(trace_len, 1), dtype=np.int32)
    tst = np.zeros(3 * max(trace_len, 1))
    sc = s._c()
    lib().or_solve(C.byref(Q.c), C.byref(A.c), _p(b), _p(c), C.byref(sc), _p(x0), _p(y0), _p(x), _p(y),
                   _p(info), trace_len, _p(tx), _p(ty), _p(txa), _p(tya), _p(tc), _p(tst),
                   None if orig is None else C.byref(orig))
    r = Result(x, y, int(info[0]), int(info[1]), int(info[2]), int(info[3]), bool(info[4]), *info[5:12].tolist(),
               rejections=int(info[12]))
    if trace_len:
        k = min(trace_len, r.iters)
        r.trace_x = tx[: k * n].reshape(k, n)
        r.trace_y = ty[: k * m].reshape(k, m)
        r.trace_xa = txa[: k * n].reshape(k, n)
        r.trace_ya = tya[: k * m].reshape(k, m)
        r.trace_cg = tc[:k].copy()
        r.trace_step = tst[: 3 * k].reshape(k, 3)
    return r
