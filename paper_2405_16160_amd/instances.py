"""Seeded synthetic QP instances  min 1/2 x'Qx + c'x  s.t.  Ax <= b  (problem (1), Sec. 1).

Every generator returns a :class:`QP` whose matrices are CSR arrays
(``rowptr`` int64, ``col`` int32 sorted within each row, ``val`` float64) with Q
stored as both triangles and exactly symmetric.  Nothing here runs any step of
PDHCG: the module only draws random data, so that the CPU reference and the GPU
library are fed from the same seeds without sharing any of the method's
arithmetic.  Seeds are ``numpy.random.default_rng([family_id, instance_id])``.

Families (the shapes of the paper's synthetic experiments, Sec. 5.1):

* ``random_qp``      Q = R'R + 1e-2 I with sparse Gaussian R, sparse Gaussian A,
                     b = A x0 + U[0,1]  (the "Random QP" family, Table 5 shape);
* ``powerlaw_qp``    power-law row lengths in A, Q = diag + signed-edge Laplacian;
* ``portfolio_qp``   Q = F F' + diag(d), 1'x = 1 as a +/- row pair, x >= 0
                     (the "Portfolio" family, Table 8 shape, direct form);
* ``mpc_qp``         linear MPC with dynamics as +/- row pairs and box limits
                     (the "Model Predictive Control" family, Table 9 shape);
* ``manufactured``   a chosen (x*, y*) with a chosen active set, so that the
                     exact optimum is known at any size.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    nrows: int
    ncols: int
    rowptr: np.ndarray  # int64 [nrows+1]
    col: np.ndarray     # int32 [nnz]
    val: np.ndarray     # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.nrows, self.ncols))

    @staticmethod
    def from_scipy(m) -> "CSR":
        m = sp.csr_matrix(m)
        m.sum_duplicates()
        m.sort_indices()
        return CSR(m.shape[0], m.shape[1], m.indptr.astype(np.int64), m.indices.astype(np.int32),
                   m.data.astype(np.float64))


@dataclasses.dataclass
class QP:
    Q: CSR
    A: CSR
    b: np.ndarray
    c: np.ndarray
    name: str = ""
    x_star: np.ndarray | None = None   # exact optimum when the construction fixes it
    y_star: np.ndarray | None = None

    @property
    def n(self) -> int:
        return self.Q.nrows

    @property
    def m(self) -> int:
        return self.A.nrows


def _rng(family: int, instance: int) -> np.random.Generator:
    return np.random.default_rng([family, instance])


def _sparse_gaussian(rng, nrows, ncols, density) -> sp.csr_matrix:
    """Bernoulli(density) mask with N(0,1) values, drawn as a uniform sample of
    Binomial(nrows*ncols, density) distinct positions (same law, O(nnz) memory)."""
    total = nrows * ncols
    k = int(rng.binomial(total, density))
    flat = rng.choice(total, size=k, replace=False)
    rows = flat // ncols
    cols = flat % ncols
    vals = rng.standard_normal(k)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nrows, ncols))


def _symmetrize(Q) -> sp.csr_matrix:
    Q = sp.csr_matrix(Q)
    Q = (Q + Q.T) * 0.5        # a+b == b+a in IEEE arithmetic: exactly symmetric
    Q = sp.csr_matrix(Q)
    Q.sum_duplicates()
    Q.sort_indices()
    return Q


def random_qp(n=1000, m=500, r_rows=None, q_density=0.01, a_density=0.01, reg=1e-2,
              family=1, instance=0) -> QP:
    """Random QP: Q = R'R + reg*I with R (r_rows x n) Bernoulli(q_density)
    Gaussian, A (m x n) Bernoulli(a_density) Gaussian, c ~ N(0,1),
    b = A x0 + s with x0 ~ N(0,1), s ~ U[0,1] (strictly feasible at x0).

    Defaults are the tiny FP64 case (n=1000, m=500, R 500x1000 at 1%); the large
    case is ``random_qp(100_000, 50_000, 50_000, 2e-5, 2e-4, family=2)``."""
    rng = _rng(family, instance)
    r_rows = m if r_rows is None else r_rows
    R = _sparse_gaussian(rng, r_rows, n, q_density)
    Q = _symmetrize(R.T @ R + reg * sp.identity(n, format="csr"))
    A = _sparse_gaussian(rng, m, n, a_density)
    c = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    s = rng.uniform(0.0, 1.0, m)
    b = A @ x0 + s
    return QP(CSR.from_scipy(Q), CSR.from_scipy(A), b, c, name=f"random_qp(n={n},m={m},seed={family}/{instance})")


def _powerlaw_lengths(rng, m, alpha=1.5, lo=1, hi=5000, mean=8.0):
    """Row lengths L = clip(round(xm * U^(-1/alpha)), lo, hi) (Pareto tail with
    exponent alpha), with the scale xm fixed by bisection so that E[L] = mean."""
    u = 1.0 - rng.uniform(0.0, 1.0, m)          # (0, 1]

    def lengths(xm):
        return np.clip(np.rint(xm * u ** (-1.0 / alpha)), lo, hi).astype(np.int64)

    a, b = 0.01, 100.0
    for _ in range(60):
        mid = 0.5 * (a + b)
        if lengths(mid).mean() < mean:
            a = mid
        else:
            b = mid
    return lengths(0.5 * (a + b))


def powerlaw_qp(n=2_000_000, m=1_000_000, a_mean=8.0, q_pairs_per_row=2, family=3, instance=0) -> QP:
    """Power-law QP: A rows with Pareto(1.5) lengths clipped to [1, 5000] and
    mean a_mean, columns uniform without replacement, N(0,1) values;
    Q = diag(U[0.01,1]) + sum_e w_e (e_i + s_e e_j)(e_i + s_e e_j)' over
    q_pairs_per_row*n random pairs (w_e = |N(0,1)|, s_e = +-1): PSD by
    construction, about 5 nonzeros per row.  c ~ N(0,1), b = A x0 + U[0,1]."""
    rng = _rng(family, instance)
    L = _powerlaw_lengths(rng, m, mean=a_mean)
    L = np.minimum(L, n)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(L, out=rowptr[1:])
    nnz = int(rowptr[-1])
    # columns uniform without replacement within each row: draw with
    # replacement, then redraw the duplicates until none remain
    cols = rng.integers(0, n, size=nnz)
    rowid = np.repeat(np.arange(m, dtype=np.int64), L)
    for _ in range(200):
        key = rowid * n + cols
        order = np.argsort(key, kind="stable")
        dup = np.zeros(nnz, dtype=bool)
        dup[order[1:]] = key[order[1:]] == key[order[:-1]]
        if not dup.any():
            break
        cols[dup] = rng.integers(0, n, size=int(dup.sum()))
    else:
        raise RuntimeError("powerlaw_qp: could not draw distinct columns")
    vals = rng.standard_normal(nnz)
    A = sp.csr_matrix((vals, cols.astype(np.int32), rowptr), shape=(m, n))
    A.sort_indices()
    # Q: signed-edge Laplacian plus a positive diagonal
    ne = q_pairs_per_row * n
    i = rng.integers(0, n, size=ne)
    j = rng.integers(0, n - 1, size=ne)
    j = np.where(j >= i, j + 1, j)
    w = np.abs(rng.standard_normal(ne))
    s = np.where(rng.uniform(size=ne) < 0.5, -1.0, 1.0)
    d = rng.uniform(0.01, 1.0, n)
    rows = np.concatenate([i, j, i, j, np.arange(n)])
    cls = np.concatenate([i, j, j, i, np.arange(n)])
    vv = np.concatenate([w, w, s * w, s * w, d])
    Q = _symmetrize(sp.csr_matrix((vv, (rows, cls)), shape=(n, n)))
    c = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    b = A @ x0 + rng.uniform(0.0, 1.0, m)
    return QP(CSR.from_scipy(Q), CSR.from_scipy(A), b, c, name=f"powerlaw_qp(n={n},m={m},seed={family}/{instance})")


def _portfolio_factor(instance, n, family, nmin, nmax):
    rng = _rng(family, instance)
    if n is None:
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    k = int(math.ceil(n / 10))
    F = rng.standard_normal((n, k)) / math.sqrt(n)
    d = rng.uniform(0.01, 0.1, n)
    return n, F, d, rng


def kappa_qp(kappa, n=50_000, m=50_000, a_density=1e-3, block=8, family=6, instance=0) -> QP:
    """Random QP whose Q has condition number exactly kappa (the condition
    sweep of Table 2's shape): Q = P B diag(lam) B' P' with lam log-spaced in
    [1/kappa, 1], B block diagonal with random orthogonal block x block blocks
    (QR of Gaussian blocks) and P a random permutation (block nonzeros per
    row); A (m x n) Bernoulli(a_density) Gaussian, c ~ N(0,1),
    b = A x0 + U[0,1] with x0 ~ N(0,1)."""
    rng = _rng(family, instance)
    nb = n // block
    assert nb * block == n, "n must be a multiple of block"
    lam = np.logspace(-math.log10(kappa), 0.0, n) if kappa > 1 else np.ones(n)
    lam = lam[rng.permutation(n)]
    rows, cols, vals = [], [], []
    for b0 in range(nb):
        G = rng.standard_normal((block, block))
        U, _ = np.linalg.qr(G)
        Bq = U @ np.diag(lam[b0 * block:(b0 + 1) * block]) @ U.T
        ii, jj = np.meshgrid(np.arange(block), np.arange(block), indexing="ij")
        rows.append((b0 * block + ii).ravel())
        cols.append((b0 * block + jj).ravel())
        vals.append(Bq.ravel())
    perm = rng.permutation(n)
    Q = sp.csr_matrix((np.concatenate(vals), (perm[np.concatenate(rows)], perm[np.concatenate(cols)])), shape=(n, n))
    Q = _symmetrize(Q)
    A = _sparse_gaussian(rng, m, n, a_density)
    c = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    b = A @ x0 + rng.uniform(0.0, 1.0, m)
    return QP(CSR.from_scipy(Q), CSR.from_scipy(A), b, c, name=f"kappa_qp(kappa={kappa:g},n={n},m={m})")


def portfolio_factor(instance=0, n=None, family=4, nmin=50, nmax=2000):
    """(F, d) of portfolio_qp's Q = F F' + diag(d) for the same arguments."""
    _, F, d, _ = _portfolio_factor(instance, n, family, nmin, nmax)
    return F, d


def _portfolio_rows(n):
    """A = [1'; -1'; -I] (budget equality as a +/- pair, x >= 0) and b = [1; -1; 0]."""
    rowptr = np.concatenate([[0, n, 2 * n], 2 * n + 1 + np.arange(n)]).astype(np.int64)
    col = np.concatenate([np.arange(n), np.arange(n), np.arange(n)]).astype(np.int32)
    val = np.concatenate([np.ones(n), -np.ones(n), -np.ones(n)])
    return CSR(n + 2, n, rowptr, col, val), np.concatenate([[1.0, -1.0], np.zeros(n)])


def portfolio_lowrank(instance=0, n=None, family=4, nmin=50, nmax=2000):
    """The same QP as ``portfolio_qp`` with Q left in factored form: returns
    (qp, (F, d)) where qp.Q is a placeholder n x n identity pattern that the
    factored entry points do not read (Q = F F' + diag(d)).  A, b, c are
    identical to ``portfolio_qp``'s; the dense Q is never formed."""
    n, F, d, rng = _portfolio_factor(instance, n, family, nmin, nmax)
    mu = rng.normal(0.05, 0.02, n)
    A, b = _portfolio_rows(n)
    eye = CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.ones(n))
    return QP(eye, A, b, -mu, name=f"portfolio_lowrank(n={n},seed={family}/{instance})"), (F, d)


def portfolio_qp(instance=0, n=None, family=4, nmin=50, nmax=2000) -> QP:
    """Portfolio QP in direct form: Q = F F' + diag(d) (dense), F n x ceil(n/10)
    with N(0, 1/n) entries, d ~ U[0.01, 0.1], c = -mu with mu ~ N(0.05, 0.02^2);
    rows 1'x <= 1, -1'x <= -1 (the budget equality as a +/- pair) and -x <= 0.
    n is log-uniform in [nmin, nmax] unless given."""
    n, F, d, rng = _portfolio_factor(instance, n, family, nmin, nmax)
    Qd = F @ F.T
    Qd = 0.5 * (Qd + Qd.T)
    Qd[np.diag_indices(n)] += d
    mu = rng.normal(0.05, 0.02, n)
    c = -mu
    A = sp.vstack([sp.csr_matrix(np.ones((1, n))), sp.csr_matrix(-np.ones((1, n))), -sp.identity(n, format="csr")])
    b = np.concatenate([[1.0, -1.0], np.zeros(n)])
    return QP(CSR.from_scipy(sp.csr_matrix(Qd)), CSR.from_scipy(A), b, c, name=f"portfolio_qp(n={n},seed={family}/{instance})")


@dataclasses.dataclass
class MPCFamily:
    """Fixed part of the linear-MPC family: dynamics, costs, constraint matrix.
    Only the initial state (hence b) changes between instances."""
    T: int
    nx: int
    nu: int
    Ad: np.ndarray
    Bd: np.ndarray
    Q: CSR
    A: CSR
    c: np.ndarray
    u_max: float
    x_max: float

    @property
    def n(self):
        return self.T * (self.nu + self.nx)

    def b_for(self, x_init: np.ndarray) -> np.ndarray:
        """Right-hand side for initial state x_init.  Variables are ordered
        [u_0..u_{T-1}, x_1..x_T]; rows are the dynamics as (+) and (-) blocks,
        then |u| <= u_max, then |x| <= x_max."""
        T, nx = self.T, self.nx
        rhs_dyn = np.zeros(T * nx)
        rhs_dyn[:nx] = self.Ad @ x_init           # x_1 - B u_0 = A x_init
        nu = self.nu
        return np.concatenate([rhs_dyn, -rhs_dyn,
                               np.full(2 * T * nu, self.u_max), np.full(2 * T * nx, self.x_max)])


def mpc_family(T=50, nx=20, nu=10, family=5, u_max=1.0, x_max=5.0) -> MPCFamily:
    """Random stable linear MPC family (the paper's MPC experiment shape):
    A_d = 0.95 * orthogonal factor of an N(0,1) matrix, B_d ~ N(0, 1/nu),
    stage cost x'Qs x + u'R u with Qs = P P'/nx + 0.01 I, R = 0.1 I, terminal
    cost Qs; equality dynamics as +/- inequality pairs, box limits as rows."""
    rng = _rng(family, 0)
    G = rng.standard_normal((nx, nx))
    Qo, Ro = np.linalg.qr(G)
    Qo = Qo * np.sign(np.diag(Ro))[None, :]
    Ad = 0.95 * Qo
    Bd = rng.standard_normal((nx, nu)) / math.sqrt(nu)
    P = rng.standard_normal((nx, nx))
    Qs = P @ P.T / nx + 0.01 * np.eye(nx)
    Qs = 0.5 * (Qs + Qs.T)
    Rc = 0.1 * np.eye(nu)
    nU = T * nu
    n = T * (nu + nx)
    Hblocks = [sp.csr_matrix(2.0 * Rc)] * T + [sp.csr_matrix(2.0 * Qs)] * T
    H = _symmetrize(sp.block_diag(Hblocks, format="csr"))
    # dynamics: x_{t+1} - Ad x_t - Bd u_t = 0 (x_0 = x_init moves to the rhs)
    rows, cols, vals = [], [], []
    for t in range(T):
        r0 = t * nx
        for i in range(nx):
            rows.append(r0 + i); cols.append(nU + t * nx + i); vals.append(1.0)
        for i in range(nx):
            for j in range(nu):
                rows.append(r0 + i); cols.append(t * nu + j); vals.append(-Bd[i, j])
        if t > 0:
            for i in range(nx):
                for j in range(nx):
                    rows.append(r0 + i); cols.append(nU + (t - 1) * nx + j); vals.append(-Ad[i, j])
    E = sp.csr_matrix((vals, (rows, cols)), shape=(T * nx, n))
    Iu = sp.hstack([sp.identity(nU), sp.csr_matrix((nU, T * nx))])
    Ix = sp.hstack([sp.csr_matrix((T * nx, nU)), sp.identity(T * nx)])
    A = sp.vstack([E, -E, Iu, -Iu, Ix, -Ix], format="csr")
    return MPCFamily(T, nx, nu, Ad, Bd, CSR.from_scipy(H), CSR.from_scipy(A), np.zeros(n), u_max, x_max)


def mpc_initial_state(instance: int, fam: MPCFamily, family=5) -> np.ndarray:
    """x_init ~ N(0, I), rejection-sampled to ||x_init||_2 <= x_max/0.95 so that
    u = 0 keeps every state inside the box (a strictly feasible instance)."""
    rng = _rng(family, 1 + instance)
    while True:
        x = rng.standard_normal(fam.nx)
        if np.linalg.norm(x) <= fam.x_max / 0.95 * 0.999:
            return x


def mpc_qp(instance=0, fam: MPCFamily | None = None) -> QP:
    fam = fam or mpc_family()
    x_init = mpc_initial_state(instance, fam)
    return QP(fam.Q, fam.A, fam.b_for(x_init), fam.c.copy(), name=f"mpc_qp(inst={instance})")


def lowrank_qp(n=100_000, m=50_000, k=5_000, p_density=1e-3, a_density=1e-4, family=7, instance=0,
               explicit=True):
    """Random QP with Q in low-rank form (the setting of Tables 3 and 4):
    Q = P P' + diag(d) with P (n x k) Bernoulli(p_density) N(0, 1) entries
    (each row of P at least one entry, so that no row of P P' is empty) and
    d ~ U[0.01, 0.1] (strictly convex); A (m x n) Bernoulli(a_density)
    N(0, 1); c ~ N(0, 1); b = A x0 + U[0, 1] with x0 ~ N(0, 1).  Returns
    (qp, P, d); qp.Q is the explicit P P' + diag(d) when explicit is set
    (else an empty n x n placeholder: the low-rank solve does not read it)."""
    rng = _rng(family, instance)
    P = _sparse_gaussian(rng, n, k, p_density)
    empty = np.nonzero(np.diff(P.indptr) == 0)[0]
    fill = sp.csr_matrix((rng.standard_normal(len(empty)), (empty, rng.integers(0, k, size=len(empty)))),
                         shape=(n, k))
    P = sp.csr_matrix(P + fill)
    P.sort_indices()
    d = rng.uniform(0.01, 0.1, n)
    A = _sparse_gaussian(rng, m, n, a_density)
    c = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    b = A @ x0 + rng.uniform(0.0, 1.0, m)
    if explicit:
        Q = _symmetrize(P @ P.T + sp.diags(d, format="csr"))
    else:
        Q = sp.csr_matrix((n, n))
    qp = QP(CSR.from_scipy(Q), CSR.from_scipy(A), b, c, name=f"lowrank_qp(n={n},m={m},k={k},seed={family}/{instance})")
    return qp, CSR.from_scipy(P), d


def manufactured(n=1000, m=500, q_density=0.01, a_density=0.01, active_frac=0.3, family=11,
                 instance=0, r_rows=None) -> QP:
    """A QP with a known optimum: draw Q, A as in ``random_qp``, pick x* ~ N(0,1),
    an active set S (each row w.p. active_frac) with y*_i ~ U[0.1, 1] on S and 0
    elsewhere, then set c = -(Q x* + A' y*), b_i = (A x*)_i on S and
    (A x*)_i + U[0.1, 1] off S.  Stationarity, feasibility and complementary
    slackness hold exactly at (x*, y*); with Q > 0, x* is the unique optimum."""
    rng = _rng(family, instance)
    r_rows = m if r_rows is None else r_rows
    R = _sparse_gaussian(rng, r_rows, n, q_density)
    Q = _symmetrize(R.T @ R + 1e-2 * sp.identity(n, format="csr"))
    A = _sparse_gaussian(rng, m, n, a_density)
    xs = rng.standard_normal(n)
    active = rng.uniform(size=m) < active_frac
    ys = np.where(active, rng.uniform(0.1, 1.0, m), 0.0)
    c = -(Q @ xs + A.T @ ys)
    slack = np.where(active, 0.0, rng.uniform(0.1, 1.0, m))
    b = A @ xs + slack
    return QP(CSR.from_scipy(Q), CSR.from_scipy(A), b, c, name=f"manufactured(n={n},m={m})", x_star=xs, y_star=ys)


def powerlaw_manufactured(n=2_000_000, m=1_000_000, active_frac=0.3, family=31, instance=0) -> QP:
    """The power-law set's Q and A (``powerlaw_qp`` with this family's seed)
    with a known optimum, drawn as in ``manufactured``: x* ~ N(0,1), an active
    set S (each row w.p. active_frac) with y*_i ~ U[0.1, 1] on S, c = -(Q x* +
    A' y*), b_i = (A x*)_i on S and (A x*)_i + U[0.1, 1] off S."""
    base = powerlaw_qp(n, m, family=family, instance=instance)
    rng = _rng(family, 1_000_000 + instance)
    Q, A = base.Q.to_scipy(), base.A.to_scipy()
    xs = rng.standard_normal(n)
    active = rng.uniform(size=m) < active_frac
    ys = np.where(active, rng.uniform(0.1, 1.0, m), 0.0)
    c = -(Q @ xs + A.T @ ys)
    b = A @ xs + np.where(active, 0.0, rng.uniform(0.1, 1.0, m))
    return QP(base.Q, base.A, b, c, name=f"powerlaw_manufactured(n={n},m={m})", x_star=xs, y_star=ys)


def row_scaled(qp: QP, spread=3.0, seed=3) -> QP:
    """The same QP with row i of A and b_i multiplied by exp(U[-spread, spread]):
    the same feasible set and optimum x, a badly scaled A (the case diagonal
    preconditioning is for)."""
    s = np.exp(np.random.default_rng(seed).uniform(-spread, spread, qp.m))
    A = sp.diags(s) @ qp.A.to_scipy()
    return dataclasses.replace(qp, A=CSR.from_scipy(A), b=qp.b * s, name=qp.name + f" rows x exp(U[-{spread:g},{spread:g}])",
                               x_star=qp.x_star, y_star=None if qp.y_star is None else qp.y_star / s)


def tiny_qp(n, m, instance=0, family=12) -> QP:
    """Dense tiny strictly convex QP (for brute-force active-set enumeration):
    Q = G'G + 0.1 I, A ~ N(0,1), c ~ N(0,1), b = A x0 + U[-0.5, 1] (some rows
    cut through x0 so that several constraints are active at the optimum)."""
    rng = _rng(family, instance)
    G = rng.standard_normal((n, n))
    Q = G.T @ G + 0.1 * np.eye(n)
    Q = 0.5 * (Q + Q.T)
    A = rng.standard_normal((m, n))
    c = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    b = A @ x0 + rng.uniform(-0.5, 1.0, m)
    # make sure the feasible set is non-empty: keep x0 feasible for every row
    b = np.maximum(b, A @ x0 + 1e-3)
    return QP(CSR.from_scipy(sp.csr_matrix(Q)), CSR.from_scipy(sp.csr_matrix(A)), b, c, name=f"tiny_qp({n},{m},{instance})")


def unconstrained(n=200, instance=0, family=13) -> QP:
    """m = 0: Q = R'R + 1e-2 I (R 2n x n at 5%), c ~ N(0,1)."""
    rng = _rng(family, instance)
    R = _sparse_gaussian(rng, 2 * n, n, 0.05)
    Q = _symmetrize(R.T @ R + 1e-2 * sp.identity(n, format="csr"))
    c = rng.standard_normal(n)
    A = CSR(0, n, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), np.zeros(0))
    return QP(CSR.from_scipy(Q), A, np.zeros(0), c, name=f"unconstrained(n={n})")
