"""Pins of the FP64 closure-network reference: analytic gradients against
central differences, the masked loss gradient, windows, bf16 rounding."""
import math

import numpy as np
import torch

from oracle import mlp


def test_layout():
    assert mlp.NPARAM == 64 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 16 + 16
    used = 33 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 2 + 2
    assert used == 37634


def test_gelu_matches_definition():
    z = np.linspace(-6, 6, 101)
    ref = np.array([0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in z])
    assert np.allclose(mlp.gelu(z), ref, atol=1e-15)
    h = 1e-6
    assert np.allclose(mlp.gelu_prime(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), atol=1e-8)


def test_gradients_against_central_differences():
    rng = np.random.default_rng(3)
    p = mlp.init_params(1)
    p += rng.normal(0, 0.05, p.shape)  # make biases and padded entries nonzero too
    X = np.zeros((5, 64))
    X[:, :33] = rng.uniform(0.3, 1.0, (5, 33))
    W = rng.normal(0, 1, (5, 16))
    Y, cache = mlp.forward(p, X)
    g, dX = mlp.backward(p, cache, W)
    f = lambda q: float((mlp.forward(q, X)[0] * W).sum())
    idx = rng.choice(len(p), 300, replace=False)
    for n, (o, s) in mlp.OFFSETS.items():  # at least 3 entries of every block
        idx = np.concatenate([idx, o + rng.choice(int(np.prod(s)), 3, replace=False)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (f(p + e) - f(p - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    fx = lambda Xq: float((mlp.forward(p, Xq)[0] * W).sum())
    for (b, j) in [(0, 0), (2, 17), (4, 32), (1, 40)]:
        E = np.zeros_like(X)
        E[b, j] = h
        fd = (fx(X + E) - fx(X - E)) / (2 * h)
        assert abs(fd - dX[b, j]) <= 1e-6 * max(1.0, abs(fd))


def test_masked_mse_gradient():
    rng = np.random.default_rng(4)
    Y = rng.normal(size=(7, 16))
    T = rng.normal(size=(7, 2))
    M = (rng.uniform(size=(7, 2)) > 0.3).astype(float)
    L, dY = mlp.masked_mse(Y, T, M)
    h = 1e-7
    for (i, j) in [(0, 0), (3, 1), (6, 0), (2, 5)]:
        E = np.zeros_like(Y)
        E[i, j] = h
        fd = (mlp.masked_mse(Y + E, T, M)[0] - mlp.masked_mse(Y - E, T, M)[0]) / (2 * h)
        assert abs(fd - dY[i, j]) <= 1e-7


def test_adam_first_step_is_signed_lr():
    p = np.zeros(4)
    g = np.array([1.0, -2.0, 0.5, 0.0])
    q, m, v = mlp.adam(p, np.zeros(4), np.zeros(4), g, 1, lr=1e-3)
    assert np.allclose(q[:3], -1e-3 * np.sign(g[:3]), rtol=1e-6) and q[3] == 0


def test_windows_replicate_padding():
    e = np.arange(10, dtype=float)
    X = mlp.windows(e)
    assert X.shape == (10, 64)
    assert np.all(X[:, 33:] == 0)
    assert np.all(X[0, :17] == 0) and X[0, 17] == 1 and X[0, 32] == 9
    assert X[5, 16] == 5 and X[5, 0] == 0 and X[5, 32] == 9
    assert np.all(X[9, 16:33] == 9)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.normal(size=1000), rng.uniform(-1e-3, 1e-3, 1000), [0.0, 1.0, -2.5, 3.0078125]])
    t = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(a), t)


def test_closure_map():
    Y = np.zeros((3, 16))
    Y[:, 0] = [0.0, math.log(2.0), -1.0]
    Y[:, 1] = [0.0, 20.0, -20.0]
    nue, drag = mlp.closure(Y, np.zeros(3), 0.1)
    assert np.allclose(nue, [0.1, 0.2, 0.1 * math.exp(-1)])
    assert np.allclose(drag, [math.log(2.0), 20.0 + math.log1p(math.exp(-20)), math.log1p(math.exp(-20))])
    nue, drag = mlp.closure(Y, np.array([1.0, 0.5, 1.0]), 0.1)
    assert nue[0] == 0.1 and nue[2] == 0.1 and drag[0] == 0 and drag[2] == 0
    assert np.isclose(nue[1], 0.1 * math.sqrt(2.0)) and np.isclose(drag[1], 0.5 * (20.0 + math.log1p(math.exp(-20))))
