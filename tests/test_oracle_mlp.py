"""Pins of the FP64 network reference (CPU): analytic gradients against central
finite differences on a 3-layer toy, closed forms of a linear layer and of
Adam's first step, and bfloat16 rounding against its definition."""
import numpy as np
import pytest

from oracle import mlp_oracle as M


def toy(seed=0, dims=(5, 7, 6, 4), B=9):
    rng = np.random.default_rng(seed)
    params = []
    for a, b in zip(dims[:-1], dims[1:]):
        params += [rng.standard_normal((a, b)) / np.sqrt(a), 0.1 * rng.standard_normal(b)]
    X = rng.standard_normal((B, dims[0]))
    T = rng.standard_normal((B, dims[-1]))
    return params, X, T


def test_gradients_match_central_differences():
    params, X, T = toy()
    loss, grads = M.loss_and_grads(params, X, T)
    h = 1e-6
    for pi, p in enumerate(params):
        it = np.nditer(p, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            orig = p[idx]
            p[idx] = orig + h
            lp = M.mse(M.forward(params, X)[-1], T)
            p[idx] = orig - h
            lm = M.mse(M.forward(params, X)[-1], T)
            p[idx] = orig
            fd = (lp - lm) / (2 * h)
            assert grads[pi][idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_single_linear_layer_closed_form():
    """One linear layer: L = mean((XW + b - T)^2) has dL/dW = 2 X'(XW + b - T)/(B n)."""
    rng = np.random.default_rng(1)
    X, W, b, T = rng.standard_normal((8, 3)), rng.standard_normal((3, 2)), rng.standard_normal(2), rng.standard_normal((8, 2))
    loss, g = M.loss_and_grads([W, b], X, T)
    R = X @ W + b - T
    assert loss == pytest.approx(np.mean(R ** 2), rel=1e-14)
    assert np.allclose(g[0], 2 * X.T @ R / R.size, rtol=1e-13)
    assert np.allclose(g[1], 2 * R.sum(axis=0) / R.size, rtol=1e-13)


def test_relu_blocks_gradient_of_dead_units():
    params, X, T = toy(2)
    params[1][:] = -100.0          # every first-layer unit dead
    loss, g = M.loss_and_grads(params, X, T)
    assert np.all(g[0] == 0) and np.all(g[1] == 0)


def test_adam_first_step_is_signed_lr():
    """After one step from zero moments, m_hat = g and v_hat = g^2, so the
    update is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    p = [rng.standard_normal((4, 3))]
    g = [rng.standard_normal((4, 3))]
    newp, st = M.adam_step(p, g, M.adam_init(p), lr=0.01)
    assert np.allclose(newp[0], p[0] - 0.01 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-12)
    assert st[0] == 1


def test_round_bf16_definition():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, 3.14159, -2.5e-3, 0.0])
    r = M.round_bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                        # tie -> even (mantissa ...0)
    assert r[2] == 1.0 + 4 * 2 ** -8          # tie -> even (rounds up to ...0)
    assert r[3] == 1.0                        # below half an ulp
    assert abs(r[4] - 3.14159) <= 2 ** -8 * 2 and r[6] == 0.0
    assert np.all(np.abs(r - vals) <= np.abs(vals) * 2 ** -8 + 1e-300)
