"""Plain NumPy multilayer perceptron: forward pass, backward pass, mean-squared
loss and one Adam step, used to check the preconditioner network's kernels.

TEST INFRASTRUCTURE ONLY (see the package header).  Project addition: the
paper has no learned preconditioner.

Network: y = W_L^T ... relu(W_1^T x + b_1) ... + b_L, i.e. layer l maps a row
x of width d_{l-1} to x @ W_l + b_l with W_l of shape [d_{l-1}, d_l], ReLU on
every layer but the last.  Parameters are packed as one flat vector, layer by
layer: W_l row-major, then b_l.

`quant` (optional) is applied to every matrix-product operand (inputs,
weights, hidden activations, back-propagated signals) to model reduced-
precision storage; `bf16_round` is round-to-nearest-even to bfloat16 (the
top 16 bits of the IEEE float32 pattern, ties to even).

Pins: central differences of the loss in FP64 (`test_oracle_mlp.py`), the
closed forms of a one-layer (affine) network and of a network whose hidden
units are all active (a product of matrices).
"""
from __future__ import annotations

import numpy as np


def n_params(dims):
    return int(sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1)))


def unpack(theta, dims):
    """Flat parameter vector -> list of (W [d_in, d_out], b [d_out])."""
    out, o = [], 0
    for i in range(len(dims) - 1):
        k, n = dims[i], dims[i + 1]
        W = theta[o:o + k * n].reshape(k, n)
        o += k * n
        b = theta[o:o + n]
        o += n
        out.append((W, b))
    assert o == theta.size
    return out


def bf16_round(a):
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64 holding the rounded value."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(a):
    return np.asarray(a, dtype=np.float64)


def forward(theta, dims, X, quant=None):
    """Returns the output [B, d_L] and the per-layer cache for backward."""
    q = quant or _ident
    layers = unpack(np.asarray(theta, dtype=np.float64), dims)
    h = np.asarray(X, dtype=np.float64)
    cache = []
    for i, (W, b) in enumerate(layers):
        hq, Wq = q(h), q(W)
        z = hq @ Wq + b
        last = i == len(layers) - 1
        a = z if last else np.maximum(z, 0.0)
        cache.append((hq, Wq, a, last))
        h = a
    return h, cache


def backward(dims, cache, dY, quant=None):
    """Gradient of a scalar loss with respect to the flat parameters and to
    the input, given dY = dLoss/dY."""
    q = quant or _ident
    grads = []
    g = np.asarray(dY, dtype=np.float64)
    dX = None
    for i in range(len(cache) - 1, -1, -1):
        hq, Wq, a, last = cache[i]
        if not last:
            g = g * (a > 0.0)
        gq = q(g)
        dW = hq.T @ gq
        db = g.sum(axis=0)
        grads.append((dW, db))
        g = gq @ Wq.T
        dX = g
    flat = []
    for dW, db in reversed(grads):
        flat += [dW.ravel(), db]
    return np.concatenate(flat), dX


def mse(Y, T):
    """Mean of the squared entries of Y - T and its gradient with respect to Y."""
    D = np.asarray(Y, dtype=np.float64) - T
    return float(np.mean(D * D)), 2.0 * D / D.size


def adam_step(theta, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1) at step t >= 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(dims, seed, last_scale=1.0):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; the last layer
    scaled by last_scale."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(dims) - 1):
        k, n = dims[i], dims[i + 1]
        W = rng.standard_normal((k, n)) * np.sqrt(2.0 / k)
        if i == len(dims) - 2:
            W *= last_scale
        parts += [W.ravel(), np.zeros(n)]
    return np.concatenate(parts)
