"""Learned warm start for a parametric QP family (growth path of the solver).

For a family whose Q, A and c are fixed and whose b depends on a parameter
theta (here the initial state of a linear MPC problem), a network maps theta
to a predicted primal-dual pair (x, y) that restarted PDHCG starts from.  The
training targets are PDHCG's own solutions, computed by the batched solver;
the network is trained by the library's bfloat16 kernels.  A prediction never
costs accuracy: the solve that starts from it stops on the same relKKT test.

Whether predictions pay is decided per family on held-out members
(`validate`), not per instance.  The solver's per-instance fallback
(warm_fallback: a start point whose relKKT exceeds that of (0, 0) is replaced
by (0, 0)) is a poor guide for families with c = 0 such as MPC: (0, 0) is then
exactly dual feasible, so its relKKT is the primal residual alone, while any
error in a predicted dual shows up undamped in the dual residual (whose
denominator 1 + ||c|| is 1).  Predictions that start far closer to the optimum
are then rejected, so the learned path solves with warm_fallback = 0.

Data preparation on the host (numpy): the dual targets are made canonical on
each row pair that encodes an equality (a'x <= u, -a'x <= -u admits
(y+ + t, y- + t) for every t), keeping max(y+ - y-, 0) and max(y- - y+, 0),
which leaves A'y and b'y unchanged.  The two sides of a box limit are not
such a pair (b+ = b-, so a shift would change b'y; at the optimum at most one
side is active anyway).  Inputs and targets are standardised per dimension.
"""
from __future__ import annotations

import dataclasses
import numpy as np

from . import instances as I
from . import mlp as _mlp
from . import pdhcg as _pd


def pair_index(fam: I.MPCFamily):
    """Row pairs (i, j) of A with row_j = -row_i and b_j = -b_i (the dynamics
    equalities as (+) and (-) blocks, in the row order of instances.mpc_family)."""
    e = fam.T * fam.nx
    return np.arange(e), e + np.arange(e)


def canonical_duals(Y, plus, minus):
    Y = np.array(Y, dtype=np.float64, copy=True)
    d = Y[..., plus] - Y[..., minus]
    Y[..., plus] = np.maximum(d, 0.0)
    Y[..., minus] = np.maximum(-d, 0.0)
    return Y


def family_qps(fam: I.MPCFamily, ids):
    thetas = np.stack([I.mpc_initial_state(int(i), fam) for i in ids])
    qps = [I.QP(fam.Q, fam.A, fam.b_for(t), fam.c) for t in thetas]
    return thetas, qps


def solve_family(fam, ids, settings: _pd.Settings, x0s=None, y0s=None, chunk=8192, log=None):
    """Batched PDHCG solves of the family members `ids` (chunks of `chunk`);
    returns (theta, x, y, results, seconds) where seconds is the device time
    of the batched solve kernels (HIP events), packing excluded.  log(msg), if
    given, is called after each chunk."""
    thetas, qps = family_qps(fam, ids)
    xs, ys, rs = [], [], []
    secs = 0.0
    for a in range(0, len(qps), chunk):
        part = qps[a:a + chunk]
        x0 = None if x0s is None else list(x0s[a:a + chunk])
        y0 = None if y0s is None else list(y0s[a:a + chunk])
        out = _pd.solve_batch(part, settings, x0s=x0, y0s=y0)
        xs += [o[0] for o in out]
        ys += [o[1] for o in out]
        rs += [o[2] for o in out]
        secs += out[0][2]["kernel_s"]
        if log:
            log(f"solved {a + len(part)} of {len(qps)}")
    return thetas, np.stack(xs), np.stack(ys), rs, secs


@dataclasses.dataclass
class Scaler:
    mu: np.ndarray
    sd: np.ndarray

    @staticmethod
    def fit(Z):
        mu = Z.mean(axis=0)
        sd = Z.std(axis=0)
        return Scaler(mu, np.where(sd > 1e-9, sd, 1.0))

    def fwd(self, Z):
        return (Z - self.mu) / self.sd

    def inv(self, Z):
        return Z * self.sd + self.mu


class DualCode:
    """Network targets for the dual: the multiplier of each equality pair,
    lam = y+ - y- (smooth in theta), and the other rows' duals as they are;
    decoding puts y+ = max(lam, 0), y- = max(-lam, 0) and projects the rest on
    y >= 0 (the canonical form of canonical_duals)."""

    def __init__(self, m, plus, minus):
        self.m, self.plus, self.minus = m, plus, minus
        mask = np.ones(m, dtype=bool)
        mask[plus] = False
        mask[minus] = False
        self.rest = np.nonzero(mask)[0]

    @property
    def width(self):
        return len(self.plus) + len(self.rest)

    def encode(self, Y):
        return np.concatenate([Y[:, self.plus] - Y[:, self.minus], Y[:, self.rest]], axis=1)

    def decode(self, Z):
        k = len(self.plus)
        Y = np.zeros((Z.shape[0], self.m))
        Y[:, self.plus] = np.maximum(Z[:, :k], 0.0)
        Y[:, self.minus] = np.maximum(-Z[:, :k], 0.0)
        Y[:, self.rest] = np.maximum(Z[:, k:], 0.0)
        return Y


class WarmStarter:
    """theta -> (x0, y0) through the trained network (y0 >= 0 by construction)."""

    def __init__(self, net: _mlp.Network, sin: Scaler, sout: Scaler, n: int, code: DualCode):
        self.net, self.sin, self.sout, self.n, self.code = net, sin, sout, n, code
        self._dev = None

    def predict(self, thetas):
        import torch
        out = []
        B = self.net.max_batch
        for a in range(0, len(thetas), B):
            Xt = torch.tensor(self.sin.fwd(thetas[a:a + B]), dtype=torch.float32, device="cuda")
            out.append(self.net.forward(Xt).cpu().numpy().astype(np.float64))
        Z = self.sout.inv(np.concatenate(out))
        return Z[:, : self.n], self.code.decode(Z[:, self.n:])


    def predict_device(self, thetas):
        """The same start points as packed float64 device tensors (x0: rows x
        n, y0: rows x m), ready for a batch of the family's members: the
        forward pass, the de-standardisation and the dual decoding run in the
        library (pdhcg_mlp_predict_start); only the inputs (n_in values per
        row) are standardised on the host."""
        import torch
        if self._dev is None:
            def dev(a, dt):
                return torch.as_tensor(np.ascontiguousarray(a, dtype=dt), device="cuda")
            self._dev = (dev(self.sout.mu, np.float64), dev(self.sout.sd, np.float64),
                         dev(self.code.plus, np.int32), dev(self.code.minus, np.int32),
                         dev(self.code.rest, np.int32))
        mu, sd, plus, minus, rest = self._dev
        Xt = torch.tensor(self.sin.fwd(thetas), dtype=torch.float32, device="cuda")
        return self.net.predict_start(Xt, mu, sd, self.n, plus, minus, rest, self.code.m)


def validate(fam, ws: "WarmStarter", ids, settings: _pd.Settings):
    """Cold and warm batched solves of held-out family members `ids` (warm:
    the network's predictions, no per-instance fallback).  Returns a dict with
    the mean iterations and kernel seconds of both and whether warm starts
    paid (fewer mean iterations)."""
    thetas, _ = family_qps(fam, ids)
    x0, y0 = ws.predict(thetas)
    s_nf = dataclasses.replace(settings, warm_fallback=0)
    _, _, _, rc, tc = solve_family(fam, ids, s_nf)
    _, _, _, rw, tw = solve_family(fam, ids, s_nf, x0s=x0, y0s=y0)
    ic = float(np.mean([r["iters"] for r in rc]))
    iw = float(np.mean([r["iters"] for r in rw]))
    return {"cold_iters": ic, "warm_iters": iw, "cold_s": tc, "warm_s": tw, "pays": iw < ic,
            "solved": sum(r["status"] == 0 for r in rc + rw), "count": 2 * len(rc)}


def train(theta, X, Y, code: DualCode, hidden=512, epochs=300, batch=256, lr=1e-3, seed=0, log=None):
    """Train the network on theta -> [x, encoded y] with Adam on standardised
    data (cosine learning-rate decay); returns the WarmStarter and the
    per-epoch mean losses."""
    import torch
    n = X.shape[1]
    Z = np.concatenate([X, code.encode(Y)], axis=1)
    sin, sout = Scaler.fit(theta), Scaler.fit(Z)
    Xt = torch.tensor(sin.fwd(theta), dtype=torch.float32, device="cuda")
    Zt = torch.tensor(sout.fwd(Z), dtype=torch.float32, device="cuda")
    net = _mlp.Network(theta.shape[1], hidden, Z.shape[1], max_batch=batch,
                       params=_mlp.init_params(theta.shape[1], hidden, Z.shape[1], seed=seed))
    rng = np.random.default_rng(seed)
    N = len(theta)
    losses = []
    net.take_loss()   # (clear the running sum)
    for ep in range(epochs):
        # the epoch's row order, drawn on the host; the library gathers each
        # minibatch from the full device arrays and the steps queue without
        # waiting; the loss is read once per epoch
        perm = torch.tensor(rng.permutation(N).astype(np.int32), device="cuda")
        step_lr = lr * 0.5 * (1 + np.cos(np.pi * ep / epochs))   # cosine decay
        for a in range(0, N - batch + 1, batch):
            net.train_rows(Xt, Zt, perm[a:a + batch], batch, lr=float(step_lr))
        tot, cnt = net.take_loss()
        losses.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.4e}")
    return WarmStarter(net, sin, sout, n, code), losses
