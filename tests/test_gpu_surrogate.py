"""GPU checks of the surrogate network kernels (BF16 MFMA forward/backward,
Adam) against the FP64 reference network, through the C ABI.

Tolerances come from BF16 operands: each product of two BF16-rounded numbers
carries a relative error up to 2^-8, so layer outputs and gradients are
compared by relative Frobenius norm <= 3e-2."""
import os
import sys
import tempfile

import numpy as np
import pytest
import torch

from oracle import mlp
from paper_2312_05647_amd import mjp, synth

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

IN, WIDTH, DEPTH = 4, 256, 3


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.fixture
def net():
    s = mjp.mjp_surrogate_create(IN, WIDTH, DEPTH, seed=synth.SEED_MLP)
    yield s
    mjp.mjp_surrogate_destroy(s)


def test_param_count_and_roundtrip(net):
    assert mjp.mjp_surrogate_num_params(net) == 133121
    p = mjp.mjp_surrogate_get_params(net)
    bound = 1 / np.sqrt(IN)
    assert np.abs(p[:IN * WIDTH]).max() <= bound
    q = synth.rng(3).normal(scale=0.05, size=p.size).astype(np.float32)
    mjp.mjp_surrogate_set_params(net, q)
    assert np.array_equal(mjp.mjp_surrogate_get_params(net), q)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "s.bin")
        mjp.mjp_surrogate_save(net, path)
        s2 = mjp.mjp_surrogate_load(path)
        try:
            assert np.array_equal(mjp.mjp_surrogate_get_params(s2), q)
        finally:
            mjp.mjp_surrogate_destroy(s2)


@pytest.mark.parametrize("n", [1, 100, 1000, 5000])
def test_forward_matches_reference(net, n):
    say(f"[gpu] surrogate forward n={n}")
    p = mjp.mjp_surrogate_get_params(net)
    X = synth.rng(n).normal(size=(n, IN)).astype(np.float32)
    y = torch.empty(n, device="cuda")
    mjp.mjp_surrogate_infer(net, torch.as_tensor(X, device="cuda"), y)
    torch.cuda.synchronize()
    ref, _ = mlp.forward(mlp.unpack(p, IN, WIDTH, DEPTH), X.astype(np.float64))
    got = y.cpu().numpy().astype(np.float64)
    assert rel(got, ref) < 3e-2, rel(got, ref)


@pytest.mark.parametrize("n", [700, 3000])
def test_gradients_match_reference(net, n):
    say(f"[gpu] surrogate gradients n={n}")
    g = synth.rng(7 + n)
    p = (g.normal(scale=0.08, size=mjp.mjp_surrogate_num_params(net))).astype(np.float32)
    mjp.mjp_surrogate_set_params(net, p)
    X = g.normal(size=(n, IN)).astype(np.float32)
    t = (np.sin(X[:, 0]) + X[:, 1] * X[:, 2]).astype(np.float32)
    loss, grad = mjp.mjp_surrogate_grad(net, torch.as_tensor(X, device="cuda"), torch.as_tensor(t, device="cuda"))
    layers = mlp.unpack(p, IN, WIDTH, DEPTH)
    rloss, rgrad = mlp.loss_and_grad(layers, X.astype(np.float64), t.astype(np.float64))
    assert abs(loss - rloss) <= 2e-2 * rloss
    off = 0
    for fi, fo in mlp.layer_sizes(IN, WIDTH, DEPTH):
        for size in (fi * fo, fo):
            a, b = grad[off:off + size].astype(np.float64), rgrad[off:off + size]
            assert rel(a, b) < 3e-2, (fi, fo, size, rel(a, b))
            off += size


def test_training_reduces_loss_and_stays_consistent(net):
    say("[gpu] surrogate training")
    g = synth.rng(21)
    n = 16384
    X = g.normal(size=(n, IN)).astype(np.float32)
    t = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2] - 0.3 * X[:, 3] ** 2).astype(np.float32)
    Xd, td = torch.as_tensor(X, device="cuda"), torch.as_tensor(t, device="cuda")
    cfg = mjp.mjp_train_cfg_default(epochs=40, batch=1024, lr=2e-3, seed=5)
    losses = mjp.mjp_surrogate_train(net, Xd, td, cfg)
    say(f"    loss {losses[0]:.4f} -> {losses[-1]:.5f}")
    assert losses[-1] < 0.05 * losses[0]
    assert np.all(np.isfinite(losses))
    p = mjp.mjp_surrogate_get_params(net)
    y = torch.empty(n, device="cuda")
    mjp.mjp_surrogate_infer(net, Xd, y)
    torch.cuda.synchronize()
    ref, _ = mlp.forward(mlp.unpack(p, IN, WIDTH, DEPTH), X.astype(np.float64))
    assert rel(y.cpu().numpy().astype(np.float64), ref) < 3e-2
    # deterministic: same seed and data -> same parameters
    s2 = mjp.mjp_surrogate_create(IN, WIDTH, DEPTH, seed=synth.SEED_MLP)
    try:
        mjp.mjp_surrogate_train(s2, Xd, td, cfg)
        assert np.array_equal(mjp.mjp_surrogate_get_params(s2), p)
    finally:
        mjp.mjp_surrogate_destroy(s2)


def test_bad_arguments(net):
    with pytest.raises(mjp.MjpError):
        mjp.mjp_surrogate_set_params(net, np.zeros(10, np.float32))
    bad = mjp.mjp_surrogate_get_params(net)
    bad[5] = np.nan
    with pytest.raises(mjp.MjpError):
        mjp.mjp_surrogate_set_params(net, bad)
    X = torch.zeros((10, IN), device="cuda")
    with pytest.raises(mjp.MjpError):
        mjp.mjp_surrogate_train(net, X, torch.zeros(10, device="cuda"), mjp.mjp_train_cfg_default(batch=100))


def test_adam_update_matches_reference():
    """Two training steps on one minibatch holding all rows; after each, the
    FP32 master parameters are compared entry by entry with the FP64 Adam
    update (oracle.mlp.adam_step, Kingma and Ba Algorithm 1 with decoupled
    decay) applied to the gradient mjp_surrogate_grad returns at the same
    parameters.  eps = 1e-3 keeps m_hat / (sqrt(v_hat) + eps) away from
    sign(g), so the comparison sees the moments and the bias correction.
    Bar: the training step sums the same rows in a shuffled order (FP32
    sums, relative ~1e-6 of each gradient), and the update's derivative in g
    is at most lr / eps = 1, so entries agree to 2e-6 + 1e-6 |w|."""
    s = mjp.mjp_surrogate_create(IN, 64, 2, seed=1)
    try:
        g = synth.rng(21)
        n = 300
        p0 = mjp.mjp_surrogate_get_params(s)
        x = torch.as_tensor(g.standard_normal((n, IN)), dtype=torch.float32, device="cuda").contiguous()
        y = torch.as_tensor(g.standard_normal(n), dtype=torch.float32, device="cuda").contiguous()
        lr, b1, b2, eps, wd = 1e-3, 0.9, 0.999, 1e-3, 0.01
        cfg = mjp.mjp_train_cfg_default(epochs=1, batch=512, lr=lr, beta1=b1, beta2=b2, eps_adam=eps,
                                        weight_decay=wd, seed=5)
        m = np.zeros(p0.size)
        v = np.zeros(p0.size)
        w = p0.astype(np.float64)
        for t in (1, 2):
            _, grad = mjp.mjp_surrogate_grad(s, x, y)
            mjp.mjp_surrogate_train(s, x, y, cfg)
            got = mjp.mjp_surrogate_get_params(s).astype(np.float64)
            ref, m, v = mlp.adam_step(w, grad, m, v, t, lr, b1, b2, eps, wd)
            err = np.abs(got - ref)
            bar = 2e-6 + 1e-6 * np.abs(ref)
            say(f"[gpu] adam step {t}: max |w_gpu - w_ref| {err.max():.2e}, moved {np.abs(ref - w).max():.2e}")
            assert (err <= bar).all(), (t, int(np.argmax(err - bar)), float(err.max()))
            assert np.abs(ref - w).max() > 1e-4  # the step is not vacuous
            w = got
    finally:
        mjp.mjp_surrogate_destroy(s)
