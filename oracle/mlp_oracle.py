"""FP64 reference of the warm-start network: a multilayer perceptron with ReLU
hidden layers and a linear output, trained on mean squared error with Adam.

TEST INFRASTRUCTURE ONLY: the GPU network kernels are checked against this
module; the product never imports it.  Written for reading: one matrix
product per layer, gradients by the chain rule in the order they are
derived, no fusion.

Parameters are a list [W1, b1, W2, b2, ..., WL, bL] with W_l of shape
(fan_in, fan_out) so that layer l maps a row batch H (B x fan_in) to
H W_l + b_l.
"""
from __future__ import annotations

import numpy as np


def forward(params, X):
    """Returns the list of layer outputs [H0 = X, H1, ..., HL]; hidden layers
    are ReLU(H W + b), the last layer is linear."""
    H = [np.asarray(X, dtype=np.float64)]
    L = len(params) // 2
    for l in range(L):
        W, b = params[2 * l], params[2 * l + 1]
        Z = H[-1] @ W + b
        H.append(np.maximum(Z, 0.0) if l < L - 1 else Z)
    return H


def mse(out, T):
    """Mean over all entries of (out - T)^2."""
    return float(np.mean((out - T) ** 2))


def loss_and_grads(params, X, T):
    """MSE loss and its gradient with respect to every parameter.
    dL/dout = 2 (out - T) / (B * n_out); back through the linear output, then
    through each ReLU layer (derivative 1 where the layer's output is > 0)."""
    H = forward(params, X)
    out = H[-1]
    B, n_out = out.shape
    G = 2.0 * (out - T) / (B * n_out)
    L = len(params) // 2
    grads = [None] * len(params)
    for l in range(L - 1, -1, -1):
        W = params[2 * l]
        grads[2 * l] = H[l].T @ G
        grads[2 * l + 1] = G.sum(axis=0)
        if l > 0:
            G = (G @ W.T) * (H[l] > 0.0)
    return mse(out, T), grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).  state = (t, m, v)."""
    t, m, v = state
    t += 1
    new_m, new_v, new_p = [], [], []
    for p, g, mi, vi in zip(params, grads, m, v):
        mi = beta1 * mi + (1 - beta1) * g
        vi = beta2 * vi + (1 - beta2) * g * g
        mh = mi / (1 - beta1 ** t)
        vh = vi / (1 - beta2 ** t)
        new_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        new_m.append(mi)
        new_v.append(vi)
    return new_p, (t, new_m, new_v)


def adam_init(params):
    return (0, [np.zeros_like(p) for p in params], [np.zeros_like(p) for p in params])


def round_bf16(a):
    """Round to the nearest bfloat16 (8 significant bits, ties to even), returned
    as float64: the precision the GPU network stores weights and activations in."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (u.astype(np.uint32) << 16).view(np.float32)
    return np.where(np.isnan(a32), np.float32(np.nan), out).astype(np.float64)
