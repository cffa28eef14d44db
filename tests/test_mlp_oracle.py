"""Pins of the FP64 network oracle: gradients against central finite
differences, softmax normalisation, GELU against its definition."""
import math

import numpy as np

from oracle import mlp


def small_params(seed=0):
    # same architecture, narrower layers so that finite differences are cheap
    return mlp.init_params(n_in=7, hidden=6, n_out=5, seed=seed)


def batch(seed=1, B=4, n_in=7, n_out=5):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, n_in))
    p = rng.random((B, n_out))
    p /= p.sum(axis=1, keepdims=True)
    t = rng.random(B)
    return x, p, t


def test_gelu_matches_normal_cdf_definition():
    for x in (-3.0, -0.7, 0.0, 0.4, 2.5):
        phi = 0.5 * (1.0 + math.erf(x / math.sqrt(2.0)))
        assert abs(mlp.gelu(np.array([x]))[0] - x * phi) < 1e-15
    x = np.linspace(-4, 4, 17)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(x)).max() < 1e-8


def test_forward_outputs_are_distributions():
    P = small_params()
    x, p, t = batch()
    q, e, _ = mlp.forward(P, x)
    assert np.all(q > 0) and np.allclose(q.sum(axis=1), 1.0, atol=1e-15)
    assert np.all(e > 0)


def test_gradients_match_central_differences():
    P = small_params(3)
    x, p, t = batch(4)
    G = mlp.backward(P, x, p, t, lam=0.7)
    h = 1e-6
    for k, W in P.items():
        it = np.nditer(W, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            old = W[idx]
            W[idx] = old + h
            lp = mlp.loss(P, x, p, t, lam=0.7)
            W[idx] = old - h
            lm = mlp.loss(P, x, p, t, lam=0.7)
            W[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - G[k][idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, G[k][idx])


def test_adam_first_step_moves_by_learning_rate():
    # with bias correction the first Adam step is lr * sign(g) (for |g| >> eps)
    P = {"w": np.array([1.0, -2.0, 3.0])}
    G = {"w": np.array([0.5, -4.0, 1e-3])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    mlp.adam_step(P, G, m, v, step=1, lr=0.1, eps=1e-12)
    assert np.allclose(P["w"], [0.9, -1.9, 2.9], atol=1e-9)
