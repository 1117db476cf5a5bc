"""GPU warm-start network (bfloat16 MFMA kernels, through the C ABI) against
the FP64 CPU reference in oracle/mlp_oracle.py.

Tolerances follow from bfloat16 storage: weights, inputs and the hidden
activations are rounded to 8 significant bits (unit roundoff u = 2^-8), so a
forward pass evaluated by the reference at the same rounded weights and
inputs differs by a few u relative to the activation scale; gradients are
compared by relative Frobenius error (<= 3e-2) and cosine (>= 0.999)."""
import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2405_16160_amd import mlp  # noqa: E402


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("dims,B", [((20, 64, 96), 32), ((20, 512, 700), 130), ((7, 33, 5), 3)])
def test_forward_and_gradients_match_reference(dims, B):
    n_in, n_hid, n_out = dims
    say(f"[mlp] dims={dims} batch={B}")
    rng = np.random.default_rng(5)
    params = mlp.init_params(n_in, n_hid, n_out, seed=1)
    params = [p + (0.05 * rng.standard_normal(p.shape) if p.ndim == 1 else 0) for p in params]
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    net = mlp.Network(n_in, n_hid, n_out, max_batch=256, params=params)
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    Tt = torch.tensor(T, dtype=torch.float32, device="cuda")
    out = net.forward(Xt).cpu().numpy().astype(np.float64)
    # reference at the bfloat16-rounded weights and inputs the kernels use
    pr = [M.round_bf16(p) if p.ndim == 2 else p for p in params]
    ref = M.forward(pr, M.round_bf16(X))[-1]
    e = rel(out, ref)
    say(f"  forward rel err {e:.2e}")
    assert e < 2e-2
    loss, grads = net.loss_grad(Xt, Tt, want_grads=True)
    rloss, rgrads = M.loss_and_grads(pr, M.round_bf16(X), T)
    assert loss == pytest.approx(rloss, rel=2e-2)
    for k, (g, r) in enumerate(zip(grads, rgrads)):
        er = rel(g, r)
        cos = float(np.dot(g.ravel(), r.ravel()) / (np.linalg.norm(g) * np.linalg.norm(r) + 1e-300))
        say(f"  grad {k} shape={r.shape} rel={er:.2e} cos={cos:.6f}")
        assert er < 3e-2 and cos > 0.999
    net.close()


def test_adam_steps_follow_reference_and_reduce_loss():
    n_in, n_hid, n_out, B = 12, 48, 20, 64
    say("[mlp] 3 Adam steps against the reference")
    rng = np.random.default_rng(8)
    params = mlp.init_params(n_in, n_hid, n_out, seed=3)
    X = rng.standard_normal((B, n_in))
    W = rng.standard_normal((n_in, n_out))
    T = np.tanh(X @ W)
    net = mlp.Network(n_in, n_hid, n_out, max_batch=B, params=params)
    Xt = torch.tensor(X, dtype=torch.float32, device="cuda")
    Tt = torch.tensor(T, dtype=torch.float32, device="cuda")
    st = M.adam_init(params)
    p = [q.copy() for q in params]
    for _ in range(3):
        net.train_step(Xt, Tt, lr=1e-3)
        _, g = M.loss_and_grads(p, X, T)
        p, st = M.adam_step(p, g, st, lr=1e-3)
    got = net.get_params()
    for a, b, p0 in zip(got, p, params):
        # the step sizes are lr-bounded; compare the movement from the start
        assert rel(a - p0, b - p0) < 0.1
    losses = [net.train_step(Xt, Tt, lr=3e-3) for _ in range(300)]
    say(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.2 * losses[0]
    net.close()


def test_queued_training_steps_equal_the_synchronous_ones():
    """pdhcg_mlp_train_step on rows picked by an index array (gathered by the
    library) takes exactly the steps of pdhcg_mlp_loss_grad + adam_step on the
    same rows gathered beforehand, and pdhcg_mlp_take_loss returns the sum of
    the step losses; shapes with no 8-aligned stride exercise the element-wise
    staging of the matrix products."""
    for dims, N, B in (((20, 512, 700), 600, 128), ((7, 33, 5), 40, 9)):
        n_in, n_hid, n_out = dims
        say(f"[mlp] queued steps dims={dims} rows={N} batch={B}")
        rng = np.random.default_rng(11)
        params = mlp.init_params(n_in, n_hid, n_out, seed=4)
        Xt = torch.tensor(rng.standard_normal((N, n_in)), dtype=torch.float32, device="cuda")
        Tt = torch.tensor(rng.standard_normal((N, n_out)), dtype=torch.float32, device="cuda")
        a = mlp.Network(n_in, n_hid, n_out, max_batch=B, params=params)
        b = mlp.Network(n_in, n_hid, n_out, max_batch=B, params=params)
        b.take_loss()
        losses = []
        for step in range(4):
            idx = torch.tensor(rng.permutation(N)[:B].astype(np.int32), device="cuda")
            losses.append(a.train_step(Xt[idx.long()].contiguous(), Tt[idx.long()].contiguous(), lr=1e-3))
            b.train_rows(Xt, Tt, idx, B, lr=1e-3)
            torch.cuda.synchronize()
        tot, cnt = b.take_loss()
        assert cnt == 4
        assert tot == pytest.approx(sum(losses), rel=1e-6)
        for pa, pb in zip(a.get_params(), b.get_params()):
            assert np.array_equal(pa, pb)
        a.close()
        b.close()


def test_device_start_points_equal_the_host_decoding():
    """pdhcg_mlp_predict_start (forward pass, de-standardisation and dual
    decoding on the device, in chunks of max_batch rows) returns exactly the
    x0, y0 of the host path (the same forward passes, then numpy: Z * sd + mu,
    y+ = max(lam, 0), y- = max(-lam, 0), the other rows max(v, 0)), for a batch
    of 150 rows over a workspace of 64; sizes that do not add up are rejected."""
    from paper_2405_16160_amd import pdhcg, warmstart as W
    say("[mlp] start points decoded on the device, 150 rows in chunks of 64")
    rng = np.random.default_rng(11)
    n_in, n_hid, n, n_pair, n_rest = 6, 64, 40, 12, 30
    m = 2 * n_pair + n_rest
    n_out = n + n_pair + n_rest
    net = mlp.Network(n_in, n_hid, n_out, max_batch=64, params=mlp.init_params(n_in, n_hid, n_out, seed=3))
    perm = rng.permutation(m)
    code = W.DualCode(m, np.sort(perm[:n_pair]), np.sort(perm[n_pair:2 * n_pair]))
    sin = W.Scaler(rng.standard_normal(n_in), rng.uniform(0.5, 2.0, n_in))
    sout = W.Scaler(rng.standard_normal(n_out), rng.uniform(0.1, 3.0, n_out))
    ws = W.WarmStarter(net, sin, sout, n, code)
    th = rng.standard_normal((150, n_in))
    xh, yh = ws.predict(th)
    xd, yd = ws.predict_device(th)
    assert xd.shape == (150, n) and yd.shape == (150, m)
    assert np.array_equal(xd.cpu().numpy(), xh)
    assert np.array_equal(yd.cpu().numpy(), yh)
    assert np.all(yh >= 0.0) and np.any(yh > 0.0)
    mu, sd, plus, minus, rest = ws._dev
    Xt = torch.tensor(sin.fwd(th), dtype=torch.float32, device="cuda")
    with pytest.raises(pdhcg.PdhcgError):
        net.predict_start(Xt, mu, sd, n + 1, plus, minus, rest, m)
    net.close()
