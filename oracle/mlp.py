"""Float64 reference of the small MLP that seeds the lead iteration.

The paper's outlook (Section IV) proposes machine learning to avoid expensive
first-principles steps; here a 3-layer perceptron maps per-mode lead features
to a guess of the surface Green's function that seeds the decimation.  This
module is the reference for the GPU training and inference kernels:
forward pass, hand-written backward pass of the mean-squared error, and Adam
(Kingma & Ba 2015, Algorithm 1), all in float64.

Network:  Z1 = X W1 + b1, A1 = tanh(Z1); Z2 = A1 W2 + b2, A2 = tanh(Z2);
          Y = A2 W3 + b3.  Weights are stored [fan_in, fan_out] row-major.
Loss:     L = mean over all n*out entries of (Y - T)^2.
"""
from __future__ import annotations

import math

import numpy as np

PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def init_params(n_in: int, width: int = 256, n_out: int = 2, seed: int = 0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    r = np.random.Generator(np.random.PCG64(seed))
    shapes = [(n_in, width), (width, width), (width, n_out)]
    p = {}
    for k, (fi, fo) in enumerate(shapes, start=1):
        lim = 1.0 / math.sqrt(fi)
        p[f"W{k}"] = r.uniform(-lim, lim, size=(fi, fo))
        p[f"b{k}"] = np.zeros(fo)
    return p


def forward(p, X):
    Z1 = X @ p["W1"] + p["b1"]
    A1 = np.tanh(Z1)
    Z2 = A1 @ p["W2"] + p["b2"]
    A2 = np.tanh(Z2)
    Y = A2 @ p["W3"] + p["b3"]
    return Y, (X, A1, A2)


def mse(Y, T) -> float:
    return float(np.mean((Y - T) ** 2))


def backward(p, cache, Y, T):
    """Gradients of the MSE with respect to every parameter (chain rule by hand)."""
    X, A1, A2 = cache
    n_el = Y.size
    dY = 2.0 * (Y - T) / n_el
    g = {}
    g["W3"] = A2.T @ dY
    g["b3"] = dY.sum(axis=0)
    dA2 = dY @ p["W3"].T
    dZ2 = dA2 * (1.0 - A2 * A2)
    g["W2"] = A1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dA1 = dZ2 @ p["W2"].T
    dZ1 = dA1 * (1.0 - A1 * A1)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam_init(p):
    return ({k: np.zeros_like(v) for k, v in p.items()}, {k: np.zeros_like(v) for k, v in p.items()})


def adam_step(p, g, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update with bias correction; t counts from 1.  Updates in place."""
    c1 = 1.0 - beta1 ** t
    c2 = 1.0 - beta2 ** t
    for k in p:
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mhat = m[k] / c1
        vhat = v[k] / c2
        p[k] = p[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


def numerical_grad(p, X, T, name, h=1e-6):
    """Central finite differences of the loss for one parameter array."""
    out = np.zeros_like(p[name])
    it = np.nditer(p[name], flags=["multi_index"])
    for _ in it:
        idx = it.multi_index
        old = p[name][idx]
        p[name][idx] = old + h
        lp = mse(forward(p, X)[0], T)
        p[name][idx] = old - h
        lm = mse(forward(p, X)[0], T)
        p[name][idx] = old
        out[idx] = (lp - lm) / (2 * h)
    return out
