"""FP64 reference of the surrogate network: TEST INFRASTRUCTURE ONLY.

An MLP in -> width -> ... -> width -> 1 with exact GELU(z) = z Phi(z)
between Linear layers, mean-squared-error loss, and its gradient by the chain
rule, written plainly in numpy float64.  Parameters use the packing of the C
ABI: for each layer, the weight [out x in] row-major, then the bias [out].
(The surrogate is not part of the paper; this only checks the GPU kernels.)
``adam_step`` is the Adam update of Kingma and Ba (ICLR 2015, Algorithm 1)
with decoupled weight decay (Loshchilov and Hutter, ICLR 2019) scaled by the
step size, the form the training kernel applies.
Pinned by tests/test_oracle_mlp.py against central finite differences, a
second GELU formula, and closed forms of the Adam update (a constant
gradient, a hand-derived two-step case, pure decay, the placement of eps).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf


def layer_sizes(in_dim: int, width: int, depth: int):
    sizes = []
    for l in range(depth + 1):
        fan_in = in_dim if l == 0 else width
        fan_out = 1 if l == depth else width
        sizes.append((fan_in, fan_out))
    return sizes


def unpack(params, in_dim: int, width: int, depth: int):
    params = np.asarray(params, np.float64)
    out, off = [], 0
    for fi, fo in layer_sizes(in_dim, width, depth):
        W = params[off:off + fi * fo].reshape(fo, fi)
        off += fi * fo
        b = params[off:off + fo]
        off += fo
        out.append((W, b))
    assert off == params.size
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(layers, X):
    """Returns the output column and the per-layer (input, pre-activation)."""
    h = np.asarray(X, np.float64)
    cache = []
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        cache.append((h, z))
        h = gelu(z) if l + 1 < len(layers) else z
    return h[:, 0], cache


def loss_and_grad(layers, X, t):
    """Mean squared error over the rows and its gradient (packed)."""
    y, cache = forward(layers, X)
    t = np.asarray(t, np.float64)
    n = len(t)
    e = y - t
    loss = float(np.mean(e * e))
    dz = (2.0 * e / n)[:, None]
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        h, _ = cache[l]
        gW = dz.T @ h
        gb = dz.sum(axis=0)
        grads[l] = (gW, gb)
        if l > 0:
            _, zprev = cache[l - 1]
            dz = (dz @ W) * gelu_grad(zprev)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_step(w, g, m, v, t: int, lr: float, beta1: float, beta2: float, eps: float, wd: float = 0.0):
    """One Adam step at step number t >= 1 (Kingma and Ba, Algorithm 1):
      m <- beta1 m + (1 - beta1) g           (first moment)
      v <- beta2 v + (1 - beta2) g^2         (second raw moment)
      m_hat = m / (1 - beta1^t),  v_hat = v / (1 - beta2^t)   (bias correction)
      w <- w - lr (m_hat / (sqrt(v_hat) + eps) + wd w)
    The last term is decoupled weight decay; eps is added outside the square
    root.  Returns the new (w, m, v), all float64."""
    assert t >= 1
    w = np.asarray(w, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    w_new = w - lr * (m_hat / (np.sqrt(v_hat) + eps) + wd * w)
    return w_new, m, v
