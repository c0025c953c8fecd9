"""FP64 oracle for the cost-model MLP that scores candidate fused blocks.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network (three weight layers, ReLU):
    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3
Loss over a batch of B rows: L = (1/B) sum_b (y_b - t_b)^2, with t the log of
the measured block time.  Backward pass written out by hand; Adam after
Kingma & Ba (2015) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8 and bias
correction.  Row-major shapes: X [B, d], W1 [d, H], W2 [H, H], W3 [H, 1].
"""
from __future__ import annotations

import numpy as np


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return y[:, 0], (X, z1, h1, z2, h2)


def loss(params, X, t):
    y, _ = forward(params, X)
    r = y - t
    return float(np.mean(r * r))


def backward(params, X, t):
    """Returns (loss, grads) with grads in the order of params."""
    W1, b1, W2, b2, W3, b3 = params
    y, (X, z1, h1, z2, h2) = forward(params, X)
    B = X.shape[0]
    r = y - t
    L = float(np.mean(r * r))
    dy = (2.0 / B) * r[:, None]               # [B, 1]
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dh2 = dy @ W3.T
    dz2 = dh2 * (z2 > 0)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * (z1 > 0)
    dW1 = X.T @ dz1
    db1 = dz1.sum(axis=0)
    return L, [dW1, db1, dW2, db2, dW3, db3]


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; `step` counts from 1."""
    for p, g, mm, vv in zip(params, grads, m, v):
        mm *= beta1
        mm += (1 - beta1) * g
        vv *= beta2
        vv += (1 - beta2) * g * g
        mhat = mm / (1 - beta1 ** step)
        vhat = vv / (1 - beta2 ** step)
        p -= lr * mhat / (np.sqrt(vhat) + eps)

