"""Diagonal preconditioning of the QP data in FP64 (numpy / scipy).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may use this module; the GPU library never imports it and
it imports nothing from the GPU library.

What is computed (Sec. 4, "Preprocessing"): positive diagonal matrices D1
(one entry per constraint row) and D2 (one per variable) such that the solver
works on  A~ = D1 A D2,  b~ = D1 b,  c~ = D2 c,  Q~ = D2 Q D2.  D1 and D2 come
from 10 Ruiz equilibration steps followed by one Pock-Chambolle step on the
symmetric matrix  K = [[Q, A'], [A, 0]].  A solution (x~, y~) of the scaled
problem gives  x = D2 x~,  y = D1 y~  for the original one.

Readings where the paper does not spell the steps out (the heuristic is the
one of the cited PDLP work):
  * Ruiz step: every row of K is divided by the square root of its largest
    magnitude, and so is the column with the same index (K is symmetric, so
    one factor per index); an index whose row is all zero keeps factor 1.
  * Pock-Chambolle step: exponent alpha = 1, i.e. every row (and its column)
    is divided by the square root of the row's 1-norm; zero rows keep 1.
  * The problem form A x <= b has no equality block G, so Q is not augmented.
  * The solver iterates on the scaled data, but every relKKT it uses
    (termination, the CG tolerance schedule, the restart tests) is that of
    the caller's problem at the mapped point (x, y) = (D2 x~, D1 y~): the
    progress metric of Section 4 is defined for the problem as posed.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from oracle import oracle as O


def kkt_matrix(Q, A) -> sp.csr_matrix:
    """K = [[Q, A'], [A, 0]] as an (n + m) x (n + m) CSR matrix (Sec. 4, preprocessing)."""
    Qs, As = Q.to_scipy(), A.to_scipy()
    if A.nrows == 0:
        return sp.csr_matrix(Qs)
    return sp.bmat([[Qs, As.T], [As, None]], format="csr")


def _rescale(K: sp.csr_matrix, f: np.ndarray) -> sp.csr_matrix:
    """diag(f) K diag(f), each entry multiplied by f_i * f_j."""
    K = K.tocoo()
    return sp.csr_matrix((K.data * (f[K.row] * f[K.col]), (K.row, K.col)), shape=K.shape)


def _factor(s: np.ndarray) -> np.ndarray:
    """1 / sqrt(s) where s > 0, else 1."""
    out = np.ones_like(s)
    pos = s > 0
    out[pos] = 1.0 / np.sqrt(s[pos])
    return out


def scaling(Q, A, ruiz_iters: int = 10, pock_chambolle: bool = True):
    """Return (d1, d2): the diagonals of D1 (length m) and D2 (length n)."""
    n = Q.nrows
    K = kkt_matrix(Q, A)
    d = np.ones(K.shape[0])
    for _ in range(ruiz_iters):
        f = _factor(abs(K).max(axis=1).toarray().ravel())
        K = _rescale(K, f)
        d *= f
    if pock_chambolle:
        f = _factor(np.asarray(abs(K).sum(axis=1)).ravel())
        K = _rescale(K, f)
        d *= f
    return d[n:].copy(), d[:n].copy()


def scale_qp(qp, d1: np.ndarray, d2: np.ndarray):
    """The scaled problem (Q~, A~, b~, c~) as a QP of the same type."""
    from dataclasses import replace
    Qs = qp.Q.to_scipy().tocoo()
    As = qp.A.to_scipy().tocoo()
    Qh = sp.csr_matrix((Qs.data * (d2[Qs.row] * d2[Qs.col]), (Qs.row, Qs.col)), shape=Qs.shape)
    Ah = sp.csr_matrix((As.data * (d1[As.row] * d2[As.col]), (As.row, As.col)), shape=As.shape)
    return replace(qp, Q=type(qp.Q).from_scipy(Qh), A=type(qp.A).from_scipy(Ah), b=qp.b * d1, c=qp.c * d2,
                   x_star=None, y_star=None)


def solve_scaled(qp, d1: np.ndarray, d2: np.ndarray, settings: O.Settings | None = None, x0=None, y0=None):
    """Solve qp through its copy scaled by the given D1, D2 (start points of
    the original problem are mapped as x~ = x / D2, y~ = y / D1), with every
    relKKT taken on qp itself; map the point back.

    Returns (x, y, result); the result's residuals and objectives are qp's."""
    x0s = None if x0 is None else np.asarray(x0, float) / d2
    y0s = None if y0 is None else np.asarray(y0, float) / d1
    r = O.solve(scale_qp(qp, d1, d2), settings, x0=x0s, y0=y0s, original=(qp, d1, d2))
    return d2 * r.x, d1 * r.y, r


def solve(qp, settings: O.Settings | None = None, ruiz_iters: int = 10, pock_chambolle: bool = True):
    """Scale with Ruiz + Pock-Chambolle, solve, map the point back.

    Returns (x, y, result, d1, d2); the result refers to the caller's problem."""
    d1, d2 = scaling(qp.Q, qp.A, ruiz_iters, pock_chambolle)
    x, y, r = solve_scaled(qp, d1, d2, settings)
    return x, y, r, d1, d2
