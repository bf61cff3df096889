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
