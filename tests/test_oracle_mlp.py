"""Pins for the FP64 reference network: the analytic gradient against central
finite differences of the loss, GELU against z Phi(z), and the packing."""
import numpy as np
from scipy.stats import norm

from oracle import mlp
from paper_2312_05647_amd import synth


def test_gelu_matches_normal_cdf_form():
    z = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(z), z * norm.cdf(z), rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-8)


def test_gradient_matches_finite_differences():
    in_dim, width, depth = 4, 8, 2
    sizes = mlp.layer_sizes(in_dim, width, depth)
    n_par = sum(fi * fo + fo for fi, fo in sizes)
    g = synth.rng(11)
    params = g.normal(scale=0.5, size=n_par)
    X = g.normal(size=(16, in_dim))
    t = g.normal(size=16)
    loss, grad = mlp.loss_and_grad(mlp.unpack(params, in_dim, width, depth), X, t)
    h = 1e-6
    for p in range(n_par):
        e = np.zeros(n_par)
        e[p] = h
        lp, _ = mlp.loss_and_grad(mlp.unpack(params + e, in_dim, width, depth), X, t)
        lm, _ = mlp.loss_and_grad(mlp.unpack(params - e, in_dim, width, depth), X, t)
        assert abs((lp - lm) / (2 * h) - grad[p]) < 1e-7 * max(1.0, abs(grad[p])), p


def test_layer_sizes_of_the_workload_network():
    """4 -> 256 -> 256 -> 256 -> 1: 133,121 parameters."""
    sizes = mlp.layer_sizes(4, 256, 3)
    assert sizes == [(4, 256), (256, 256), (256, 256), (256, 1)]
    assert sum(fi * fo + fo for fi, fo in sizes) == 133121


# ---- Adam (Kingma and Ba, ICLR 2015, Algorithm 1; decoupled decay) pins


def _run_adam(ws, gs, lr, b1, b2, eps, wd=0.0):
    w = np.asarray(ws, np.float64)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    out = []
    for t, g in enumerate(gs, start=1):
        w, m, v = mlp.adam_step(w, g, m, v, t, lr, b1, b2, eps, wd)
        out.append(w.copy())
    return out, m, v


def test_adam_constant_gradient_closed_form():
    """A constant gradient g from zero moments: m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so after bias correction m_hat = g, v_hat = g^2 and
    every step moves w by lr g / (|g| + eps): after t steps
    w_t = w_0 - t lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 5.0])
    w0 = np.array([1.0, -1.0, 0.5, 0.0])
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-4
    ws, m, v = _run_adam(w0, [g] * 7, lr, b1, b2, eps)
    assert np.allclose(m, (1 - b1 ** 7) * g, rtol=1e-13)
    assert np.allclose(v, (1 - b2 ** 7) * g * g, rtol=1e-13)
    for t, w in enumerate(ws, start=1):
        assert np.allclose(w, w0 - t * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_adam_two_steps_by_hand():
    """b1 = b2 = 1/2, eps = 0, lr = 1, from w = 0.  Step 1: m = g1/2,
    v = g1^2/2, both corrections 1/2, so the step is sign(g1).  Step 2: the
    corrections are 3/4, m_hat = (g1 + 2 g2)/3, v_hat = (g1^2 + 2 g2^2)/3.
    With g1 = (1, 5, 5), g2 = (-1, 1, -1): v_hat = (1, 9, 9) and m_hat =
    (-1/3, 7/3, 1), so the second step is (-1/3, 7/9, 1/3)."""
    g1 = np.array([1.0, 5.0, 5.0])
    g2 = np.array([-1.0, 1.0, -1.0])
    ws, m, v = _run_adam(np.zeros(3), [g1, g2], 1.0, 0.5, 0.5, 0.0)
    assert np.allclose(ws[0], [-1.0, -1.0, -1.0], rtol=0, atol=1e-15)
    assert np.allclose(ws[1], [-1.0 + 1.0 / 3.0, -1.0 - 7.0 / 9.0, -1.0 - 1.0 / 3.0], rtol=0, atol=1e-15)
    assert np.allclose(m, [0.25 * 1 + 0.5 * -1, 0.25 * 5 + 0.5 * 1, 0.25 * 5 + 0.5 * -1], rtol=0, atol=1e-15)
    assert np.allclose(v, [0.25 + 0.5, 0.25 * 25 + 0.5, 0.25 * 25 + 0.5], rtol=0, atol=1e-15)


def test_adam_decoupled_decay_and_eps_placement():
    """With a zero gradient only the decay acts: w <- w (1 - lr wd).  With a
    gradient at step 1 the step is lr (g / (|g| + eps) + wd w): eps sits
    outside the square root (g = 3, eps = 1: 3/4, not 3/sqrt(10))."""
    w0 = np.array([2.0, -4.0])
    ws, _, _ = _run_adam(w0, [np.zeros(2)] * 3, 0.1, 0.9, 0.999, 1e-8, wd=0.5)
    for t, w in enumerate(ws, start=1):
        assert np.allclose(w, w0 * 0.95 ** t, rtol=1e-14)
    ws, _, _ = _run_adam(np.array([1.0]), [np.array([3.0])], 1.0, 0.9, 0.999, 1.0, wd=0.25)
    assert np.allclose(ws[0], [1.0 - (0.75 + 0.25)], rtol=0, atol=1e-15)
