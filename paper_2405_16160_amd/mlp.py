"""Python binding of include/pdhcg_mlp.h (argument marshalling only): the
warm-start network whose forward, backward and Adam steps run in the
library's HIP kernels.  Inputs and targets are torch float32 device tensors."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import pdhcg as _p


def _lib():
    L = _p.lib()
    if not getattr(L, "_mlp_bound", False):
        P = C.c_void_p
        L.pdhcg_mlp_create.argtypes = [C.POINTER(P), C.c_int32, C.c_int32, C.c_int32, C.c_int32, P]
        L.pdhcg_mlp_num_params.argtypes = [P]
        L.pdhcg_mlp_num_params.restype = C.c_int64
        L.pdhcg_mlp_set_params.argtypes = [P, P]
        L.pdhcg_mlp_get_params.argtypes = [P, P]
        L.pdhcg_mlp_forward.argtypes = [P, P, C.c_int32, P]
        L.pdhcg_mlp_loss_grad.argtypes = [P, P, P, C.c_int32, P, P]
        L.pdhcg_mlp_adam_step.argtypes = [P, C.c_float, C.c_float, C.c_float, C.c_float]
        L.pdhcg_mlp_train_step.argtypes = [P, P, P, P, C.c_int32, C.c_float, C.c_float, C.c_float, C.c_float]
        L.pdhcg_mlp_take_loss.argtypes = [P, P, P]
        L.pdhcg_mlp_predict_start.argtypes = [P, P, C.c_int32, P, P, C.c_int32, C.c_int32, P, P, C.c_int32, P,
                                              C.c_int32, P, P]
        L.pdhcg_mlp_destroy.argtypes = [P]
        L.pdhcg_mlp_destroy.restype = None
        L._mlp_bound = True
    return L


MLP_EXPORTS = ["pdhcg_mlp_create", "pdhcg_mlp_num_params", "pdhcg_mlp_set_params", "pdhcg_mlp_get_params",
               "pdhcg_mlp_forward", "pdhcg_mlp_loss_grad", "pdhcg_mlp_adam_step", "pdhcg_mlp_train_step",
               "pdhcg_mlp_take_loss", "pdhcg_mlp_predict_start", "pdhcg_mlp_destroy"]


def init_params(n_in, n_hid, n_out, seed=0):
    """He-uniform weights and zero biases, drawn on the host from a seeded
    numpy generator (packed layout of pdhcg_mlp.h)."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in ((n_in, n_hid), (n_hid, n_hid), (n_hid, n_out)):
        lim = np.sqrt(6.0 / a)
        out += [rng.uniform(-lim, lim, size=(a, b)), np.zeros(b)]
    return out


def pack(params):
    return np.concatenate([np.asarray(p, dtype=np.float32).ravel() for p in params])


def unpack(vec, n_in, n_hid, n_out):
    shapes = [(n_in, n_hid), (n_hid,), (n_hid, n_hid), (n_hid,), (n_hid, n_out), (n_out,)]
    out, k = [], 0
    for s in shapes:
        cnt = int(np.prod(s))
        out.append(np.asarray(vec[k:k + cnt], dtype=np.float64).reshape(s))
        k += cnt
    return out


class Network:
    def __init__(self, n_in, n_hid, n_out, max_batch, params=None):
        import torch
        self.n_in, self.n_hid, self.n_out, self.max_batch = n_in, n_hid, n_out, max_batch
        h = C.c_void_p()
        _p._check(_lib().pdhcg_mlp_create(C.byref(h), n_in, n_hid, n_out, max_batch, _p._stream_ptr()))
        self.h = h
        _p._live.add(self)
        self.np = _lib().pdhcg_mlp_num_params(h)
        self.set_params(params if params is not None else init_params(n_in, n_hid, n_out))
        self._torch = torch

    def set_params(self, params):
        v = pack(params) if isinstance(params, (list, tuple)) else np.ascontiguousarray(params, dtype=np.float32)
        assert v.size == self.np
        _p._check(_lib().pdhcg_mlp_set_params(self.h, v.ctypes.data))

    def get_params(self):
        v = np.zeros(self.np, dtype=np.float32)
        _p._check(_lib().pdhcg_mlp_get_params(self.h, v.ctypes.data))
        return unpack(v, self.n_in, self.n_hid, self.n_out)

    def forward(self, X):
        torch = self._torch
        X = X.contiguous()
        Y = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device=X.device)
        _p._check(_lib().pdhcg_mlp_forward(self.h, X.data_ptr(), X.shape[0], Y.data_ptr()))
        return Y

    def predict_start(self, X, mu, sd, n, plus, minus, rest, m):
        """Packed start points (x0: rows x n, y0: rows x m, float64 device
        tensors) from the network's outputs on X (pdhcg_mlp_predict_start);
        mu, sd: float64 device tensors of n_out; plus, minus, rest: int32
        device tensors of rows of y."""
        torch = self._torch
        X = X.contiguous()
        rows = X.shape[0]
        x0 = torch.empty((rows, n), dtype=torch.float64, device=X.device)
        y0 = torch.empty((rows, max(m, 1)), dtype=torch.float64, device=X.device)
        _p._check(_lib().pdhcg_mlp_predict_start(self.h, X.data_ptr(), rows, mu.data_ptr(), sd.data_ptr(), n,
                                                 plus.numel(), plus.data_ptr(), minus.data_ptr(), rest.numel(),
                                                 rest.data_ptr(), m, x0.data_ptr(), y0.data_ptr()))
        return x0, y0[:, :m]

    def loss_grad(self, X, T, want_grads=False):
        loss = C.c_float()
        g = np.zeros(self.np, dtype=np.float32) if want_grads else None
        _p._check(_lib().pdhcg_mlp_loss_grad(self.h, X.contiguous().data_ptr(), T.contiguous().data_ptr(), X.shape[0],
                                             C.byref(loss), None if g is None else g.ctypes.data))
        return loss.value, (unpack(g, self.n_in, self.n_hid, self.n_out) if want_grads else None)

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        _p._check(_lib().pdhcg_mlp_adam_step(self.h, lr, beta1, beta2, eps))

    def train_step(self, X, T, lr):
        loss, _ = self.loss_grad(X, T)
        self.adam_step(lr)
        return loss

    def train_rows(self, X, T, rows, batch, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """Queue one training step on rows[0:batch] (an int32 device tensor or
        a view into one) of the full data tensors X and T; no wait."""
        _p._check(_lib().pdhcg_mlp_train_step(self.h, X.data_ptr(), T.data_ptr(), rows.data_ptr(), batch, lr,
                                              beta1, beta2, eps))

    def take_loss(self):
        """(sum of the step losses since the last call, number of steps)."""
        s, k = C.c_double(), C.c_int64()
        _p._check(_lib().pdhcg_mlp_take_loss(self.h, C.byref(s), C.byref(k)))
        return s.value, k.value

    def close(self):
        if getattr(self, "h", None):
            _lib().pdhcg_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
