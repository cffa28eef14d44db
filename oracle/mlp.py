"""FP64 oracle of the learned DOS reconstruction network.

TEST INFRASTRUCTURE (see oracle/__init__.py).  This is the reference the
GPU network kernels are checked against: the same architecture written out
with NumPy matrix products in float64, forward and backward.

Architecture (one sample x has 129 features: 128 Chebyshev moments and the
disorder strength):
    h1 = gelu(x  W1 + b1)          W1: 129 x 512
    h2 = gelu(h1 W2 + b2)          W2: 512 x 512
    h3 = gelu(h2 W3 + b3)          W3: 512 x 512
    z  = h3 W4 + b4                W4: 512 x 512   (DOS logits, 512 bins)
    q  = softmax(z)                (DOS mass per bin: non-negative, sums to 1)
    e  = softplus(h3 w5 + b5)      w5: 512 x 1     (predicted L1 error)
Loss for a batch of B samples with target bin masses p (rows sum to 1) and
target errors t:
    L = (1/B) sum_b [ -sum_k p_bk log q_bk ] + lam (1/B) sum_b (e_b - t_b)^2
GELU is the exact form x Phi(x) with Phi the standard normal CDF.
"""
from __future__ import annotations

import math

import numpy as np

try:
    from scipy.special import erf as _erf
except ImportError:  # pragma: no cover
    _erf = np.vectorize(math.erf)

SQRT1_2 = 1.0 / math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(x):
    return 0.5 * x * (1.0 + _erf(x * SQRT1_2))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + _erf(x * SQRT1_2)) + x * INV_SQRT_2PI * np.exp(-0.5 * x * x)


def softplus(x):
    return np.where(x > 20.0, x, np.log1p(np.exp(np.minimum(x, 20.0))))


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def init_params(n_in=129, hidden=512, n_out=512, seed=0):
    """He-style initialisation (float64)."""
    rng = np.random.default_rng(seed)
    dims = [n_in, hidden, hidden, hidden]
    P = {}
    for i in range(3):
        P[f"W{i + 1}"] = rng.standard_normal((dims[i], dims[i + 1])) * math.sqrt(2.0 / dims[i])
        P[f"b{i + 1}"] = np.zeros(dims[i + 1])
    P["W4"] = rng.standard_normal((hidden, n_out)) * math.sqrt(1.0 / hidden)
    P["b4"] = np.zeros(n_out)
    P["w5"] = rng.standard_normal((hidden, 1)) * math.sqrt(1.0 / hidden)
    P["b5"] = np.zeros(1)
    return P


def forward(P, x):
    """Returns (q, e, cache)."""
    cache = {"x": x}
    h = x
    for i in range(1, 4):
        a = h @ P[f"W{i}"] + P[f"b{i}"]
        cache[f"a{i}"] = a
        h = gelu(a)
        cache[f"h{i}"] = h
    z = h @ P["W4"] + P["b4"]
    z = z - z.max(axis=1, keepdims=True)
    ez = np.exp(z)
    q = ez / ez.sum(axis=1, keepdims=True)
    s = h @ P["w5"] + P["b5"]
    e = softplus(s)[:, 0]
    cache.update(q=q, s=s, e=e)
    return q, e, cache


def loss(P, x, p, t, lam=1.0):
    q, e, _ = forward(P, x)
    B = x.shape[0]
    ce = -np.sum(p * np.log(np.maximum(q, 1e-300))) / B
    mse = np.sum((e - t) ** 2) / B
    return ce + lam * mse


def backward(P, x, p, t, lam=1.0):
    """Gradients of `loss` with respect to every parameter (float64)."""
    q, e, c = forward(P, x)
    B = x.shape[0]
    G = {}
    dz = (q - p) / B                              # softmax + cross-entropy
    ds = (2.0 * lam / B) * (e - t)[:, None] * sigmoid(c["s"])
    h3 = c["h3"]
    G["W4"] = h3.T @ dz
    G["b4"] = dz.sum(axis=0)
    G["w5"] = h3.T @ ds
    G["b5"] = ds.sum(axis=0)
    dh = dz @ P["W4"].T + ds @ P["w5"].T
    for i in (3, 2, 1):
        da = dh * gelu_grad(c[f"a{i}"])
        hin = c[f"h{i - 1}"] if i > 1 else c["x"]
        G[f"W{i}"] = hin.T @ da
        G[f"b{i}"] = da.sum(axis=0)
        if i > 1:
            dh = da @ P[f"W{i}"].T
    return G


def adam_step(P, G, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected), in place on P, m, v."""
    for k in P:
        m[k] = beta1 * m[k] + (1.0 - beta1) * G[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * G[k] * G[k]
        mh = m[k] / (1.0 - beta1 ** step)
        vh = v[k] / (1.0 - beta2 ** step)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
