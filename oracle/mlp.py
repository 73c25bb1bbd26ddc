"""Float64 reference of the schedule model -- TEST INFRASTRUCTURE ONLY.

A multilayer perceptron with ReLU hidden layers predicts, for each candidate
schedule, the log of its runtime from four features of a product.  This module
is the plain definition the GPU kernels are checked against:

* forward:  h_0 = x;  h_i = relu(h_{i-1} W_i + b_i) for hidden layers;  y = h_L W_out + b_out
* loss:     L = sum over observed entries (mask = 1) of (y - target)^2 / (number observed)
* backward: the chain rule for the above, layer by layer
* Adam:     Kingma and Ba, "Adam: a method for stochastic optimization" (ICLR 2015),
            with bias-corrected first and second moments.

Parameters are a list ``[W1, b1, W2, b2, ..., Wout, bout]`` with ``W_i`` of shape
(fan_in, fan_out).  Pinned by central finite differences and closed forms in
``tests/test_oracle_mlp.py``.
"""
from __future__ import annotations

import numpy as np


def init_params(sizes, seed: int = 0):
    """He-style initialisation from a seeded numpy generator (sizes = [4, 64, 64, 64, S])."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        params.append(rng.standard_normal((fi, fo)) * np.sqrt(2.0 / fi))
        params.append(np.zeros(fo))
    return params


def forward(params, X):
    """Returns (Y, acts) where acts[i] is the input of layer i (acts[0] = X) and
    pre[i] the pre-activation of hidden layer i."""
    acts = [np.asarray(X, dtype=np.float64)]
    pre = []
    nl = len(params) // 2
    h = acts[0]
    for i in range(nl):
        W, b = params[2 * i], params[2 * i + 1]
        z = h @ W + b
        if i < nl - 1:
            pre.append(z)
            h = np.maximum(z, 0.0)
            acts.append(h)
        else:
            h = z
    return h, (acts, pre)


def loss(Y, T, M):
    cnt = max(float(M.sum()), 1.0)
    d = (Y - T) * M
    return float((d * d).sum() / cnt)


def backward(params, cache, Y, T, M):
    """Gradients of ``loss`` w.r.t. every parameter, same order as ``params``."""
    acts, pre = cache
    cnt = max(float(M.sum()), 1.0)
    g = 2.0 * (Y - T) * M / cnt          # dL/dY
    nl = len(params) // 2
    grads = [None] * len(params)
    for i in reversed(range(nl)):
        W = params[2 * i]
        grads[2 * i] = acts[i].T @ g
        grads[2 * i + 1] = g.sum(axis=0)
        if i > 0:
            g = (g @ W.T) * (pre[i - 1] > 0)
    return grads


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1).  Returns new (params, m, v)."""
    newp, newm, newv = [], [], []
    for p, g, mi, vi in zip(params, grads, m, v):
        mi = beta1 * mi + (1 - beta1) * g
        vi = beta2 * vi + (1 - beta2) * g * g
        mhat = mi / (1 - beta1 ** t)
        vhat = vi / (1 - beta2 ** t)
        newp.append(p - lr * mhat / (np.sqrt(vhat) + eps))
        newm.append(mi)
        newv.append(vi)
    return newp, newm, newv


def predict_argmin(params, X, valid=None):
    Y, _ = forward(params, X)
    if valid is not None:
        Y = np.where(valid, Y, np.inf)
    return np.argmin(Y, axis=1)
