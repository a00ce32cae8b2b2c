"""FP64 reference of the block-skip network (test infrastructure).

A multilayer perceptron 8 -> 64 -> 64 -> 1 with ReLU hidden layers predicts,
from features of a candidate output block, the logit of the probability that
the block falls under the drop threshold.  Trained with the mean binary
cross-entropy on logits and Adam.  Plain numpy, FP64, written out step by step.

Parameter vector layout (shared with the GPU kernels; 4801 floats):
W1 (64 x 8, row-major), b1 (64), W2 (64 x 64, row-major, W2[j, k] maps input
k to output j), b2 (64), w3 (64), b3 (1).
"""
from __future__ import annotations

import numpy as np

NF, NH = 8, 64
SIZES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
         ("w3", (NH,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, off = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[off:off + n].reshape(shape)
        off += n
    return out


def forward(theta, X):
    """Logits z for rows of X (n x 8)."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ p["W1"].T + p["b1"], 0.0)
    h2 = np.maximum(h1 @ p["W2"].T + p["b2"], 0.0)
    return h2 @ p["w3"] + p["b3"][0]


def softplus(z):
    return np.logaddexp(0.0, z)


def loss_and_grad(theta, X, y):
    """Mean of softplus(z) - y z over the samples, and its gradient."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = X.shape[0]
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["w3"] + p["b3"][0]
    loss = float(np.mean(softplus(z) - y * z))
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n          # d loss / d z
    g = {}
    g["w3"] = dz @ h2
    g["b3"] = np.array([dz.sum()])
    da2 = np.outer(dz, p["w3"]) * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ p["W2"]) * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    grad = np.concatenate([g[name].ravel() for name, _ in SIZES])
    return loss, grad


def adam_step(theta, m, v, grad, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; t counts from 1."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
