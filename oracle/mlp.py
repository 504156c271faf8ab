"""Energy surrogate: a perceptron with two GELU hidden layers, trained by Adam.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The learned part of the optimisation (the trial steps of the line search of
Sec. II A, Eq. OptPro, are screened by a cheap model of E) is not specified by
the paper beyond "a small network"; the network, its initialisation and its
training follow the reading stated in the design notes:

* y(x) = W3 gelu(W2 gelu(W1 x + b1) + b2) + b3, gelu(z) = z/2 (1 + erf(z/sqrt 2));
* parameters flattened in the order W1 [w][n_in], b1 [w], W2 [w][w], b2 [w],
  W3 [w], b3 [1]; each drawn uniform in +-1/sqrt(fan_in) from SplitMix64
  (Steele, Lea, Flood 2014) with counter = position in the flat vector;
* loss = mean squared error against targets standardised by their mean and
  standard deviation; Adam (Kingma and Ba) with beta = (0.9, 0.999),
  eps = 1e-8, moments reset at each refit.

Plain numpy in float64.
"""
from __future__ import annotations

import math

import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, i: int) -> int:
    """i-th output of SplitMix64 seeded with ``seed`` (counter form)."""
    z = (seed + (i + 1) * GAMMA) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def uniform_counter(seed: int, offset: int, n: int) -> np.ndarray:
    """u_i = (splitmix64(seed, offset + i) >> 11) * 2^-53 in [0, 1)."""
    return np.array([(splitmix64(seed, offset + i) >> 11) * 2.0 ** -53 for i in range(n)], dtype=np.float64)


def layout(n_in: int, width: int):
    """(name, shape, fan_in) of the flat parameter vector."""
    return [("W1", (width, n_in), n_in), ("b1", (width,), n_in), ("W2", (width, width), width), ("b2", (width,), width),
            ("W3", (width,), width), ("b3", (1,), width)]


def param_count(n_in: int, width: int) -> int:
    return sum(int(np.prod(s)) for _, s, _ in layout(n_in, width))


def init_params(n_in: int, width: int, seed: int) -> np.ndarray:
    """Flat parameters, rounded to float32 as the network stores them."""
    out, off = [], 0
    for _, shape, fan in layout(n_in, width):
        k = int(np.prod(shape))
        u = uniform_counter(seed, off, k)
        out.append(((2.0 * u - 1.0) / math.sqrt(fan)).astype(np.float32))
        off += k
    return np.concatenate(out)


def unpack(theta: np.ndarray, n_in: int, width: int):
    p, off = {}, 0
    for name, shape, _ in layout(n_in, width):
        k = int(np.prod(shape))
        p[name] = np.asarray(theta[off:off + k], dtype=np.float64).reshape(shape)
        off += k
    return p


_erf = np.vectorize(math.erf)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(theta, X, n_in, width, cache=False):
    p = unpack(theta, n_in, width)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ p["W1"].T + p["b1"]
    A1 = gelu(Z1)
    Z2 = A1 @ p["W2"].T + p["b2"]
    A2 = gelu(Z2)
    y = A2 @ p["W3"] + p["b3"][0]
    if cache:
        return y, (X, Z1, A1, Z2, A2, p)
    return y


def loss_grad(theta, X, t, n_in, width):
    """Mean squared error (1/n) sum (y - t)^2 and its gradient in the flat layout."""
    y, (X, Z1, A1, Z2, A2, p) = forward(theta, X, n_in, width, cache=True)
    n = X.shape[0]
    r = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    gW3 = A2.T @ dy
    gb3 = np.array([dy.sum()])
    dZ2 = np.outer(dy, p["W3"]) * gelu_grad(Z2)
    gW2 = dZ2.T @ A1
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ p["W2"]) * gelu_grad(Z1)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, gb3])
    return loss, g


def standardize(t):
    t = np.asarray(t, dtype=np.float64)
    mu = t.mean()
    sd = t.std()
    return mu, (sd if sd > 0 else 1.0)


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def train(theta, X, targets, n_in, width, steps, lr):
    """Full-batch Adam on standardised targets; returns (theta, (mu, sd), losses)."""
    mu, sd = standardize(targets)
    ts = (np.asarray(targets, dtype=np.float64) - mu) / sd
    theta = np.asarray(theta, dtype=np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    losses = []
    for k in range(1, steps + 1):
        loss, g = loss_grad(theta, X, ts, n_in, width)
        losses.append(loss)
        theta, m, v = adam_step(theta, g, m, v, k, lr)
    return theta, (mu, sd), losses


def predict(theta, X, n_in, width, stats=(0.0, 1.0)):
    return forward(theta, X, n_in, width) * stats[1] + stats[0]
