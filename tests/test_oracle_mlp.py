"""Pins of the oracle MLP: central differences, closed forms, bf16 rounding
against its definition, Adam against a hand-worked first step."""
import numpy as np

from oracle import mlp


def _loss(theta, dims, X, T):
    Y, _ = mlp.forward(theta, dims, X)
    return mlp.mse(Y, T)[0]


def test_backward_matches_central_differences():
    dims = [7, 5, 6, 4]
    rng = np.random.default_rng(3)
    theta = mlp.init_params(dims, 4)
    theta[dims[0] * dims[1]:dims[0] * dims[1] + dims[1]] = 0.1   # some positive biases
    X = rng.standard_normal((9, dims[0]))
    T = rng.standard_normal((9, dims[-1]))
    Y, cache = mlp.forward(theta, dims, X)
    g, dX = mlp.backward(dims, cache, mlp.mse(Y, T)[1])
    h = 1e-6
    num = np.empty_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        num[i] = (_loss(theta + e, dims, X, T) - _loss(theta - e, dims, X, T)) / (2 * h)
    assert np.max(np.abs(num - g)) < 1e-7 * max(1.0, np.max(np.abs(g)))
    # input gradient
    numx = np.empty_like(X)
    for idx in np.ndindex(*X.shape):
        e = np.zeros_like(X)
        e[idx] = h
        numx[idx] = (mlp.mse(mlp.forward(theta, dims, X + e)[0], T)[0] -
                     mlp.mse(mlp.forward(theta, dims, X - e)[0], T)[0]) / (2 * h)
    assert np.max(np.abs(numx - dX)) < 1e-7 * max(1.0, np.max(np.abs(dX)))


def test_affine_network_closed_form():
    dims = [4, 3]
    rng = np.random.default_rng(5)
    W = rng.standard_normal((4, 3))
    b = rng.standard_normal(3)
    theta = np.concatenate([W.ravel(), b])
    X = rng.standard_normal((6, 4))
    Y, cache = mlp.forward(theta, dims, X)
    assert np.allclose(Y, X @ W + b, rtol=0, atol=1e-14)
    dY = rng.standard_normal((6, 3))
    g, dX = mlp.backward(dims, cache, dY)
    assert np.allclose(g[:12].reshape(4, 3), X.T @ dY, atol=1e-13)
    assert np.allclose(g[12:], dY.sum(0), atol=1e-13)
    assert np.allclose(dX, dY @ W.T, atol=1e-13)


def test_all_active_network_is_matrix_product():
    # positive inputs and weights keep every ReLU in its linear branch
    dims = [5, 4, 3]
    rng = np.random.default_rng(6)
    W1, W2 = rng.uniform(0.1, 1, (5, 4)), rng.uniform(-1, 1, (4, 3))
    theta = np.concatenate([W1.ravel(), np.zeros(4), W2.ravel(), np.zeros(3)])
    X = rng.uniform(0.1, 1, (7, 5))
    Y, _ = mlp.forward(theta, dims, X)
    assert np.allclose(Y, X @ (W1 @ W2), atol=1e-13)


def test_bf16_round_definition():
    # exactly representable values are kept; halfway cases go to even
    assert mlp.bf16_round(1.0) == 1.0
    assert mlp.bf16_round(1.0 + 2.0 ** -8) == 1.0                 # tie, 1.0 is even
    assert mlp.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # tie, odd -> up
    assert mlp.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -12) == 1.0 + 2.0 ** -7
    x = np.random.default_rng(7).standard_normal(1000)
    r = mlp.bf16_round(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-12))   # half an ulp of 8 bits
    # 8 significant bits: r * 2^(7 - floor(log2|r|)) is an integer
    e = np.floor(np.log2(np.abs(r)))
    assert np.allclose(r * 2.0 ** (7 - e), np.round(r * 2.0 ** (7 - e)), atol=0)


def test_adam_first_step_is_signed_lr():
    # at t = 1 the bias-corrected moments are g and g^2: step = lr g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3])
    th, m, v = mlp.adam_step(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 0.01, eps=0.0)
    assert np.allclose(th, -0.01 * np.sign(g), atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
