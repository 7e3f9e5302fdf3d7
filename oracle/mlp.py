"""Float64 reference of the learned star-pressure network (test infrastructure).

Network: x (6) -> tanh(W1 x + b1) (32) -> tanh(W2 h1 + b2) (32) -> W3 h2 + b3.
Inputs are standardised with the parameter block's mean/std; the loss is the
mean squared error over a batch.  Parameter layout (flat): W1[32][6], b1[32],
W2[32][32], b2[32], W3[32], b3, mean[6], std[6].

The gradient is written out by the chain rule.  Pins (tests): the forward
pass against closed forms of single-path parameter blocks (weight layout,
standardisation, input slots), the features against a hand-computed case and
their invariances, the gradients against central differences.  The network
is not from the paper: these pins come from its definition here, not from
the paper.
"""
from __future__ import annotations

import numpy as np

NW = 1313


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    W1 = P[0:192].reshape(32, 6)
    b1 = P[192:224]
    W2 = P[224:1248].reshape(32, 32)
    b2 = P[1248:1280]
    W3 = P[1280:1312]
    b3 = P[1312]
    mean = P[1313:1319]
    std = P[1319:1325]
    return W1, b1, W2, b2, W3, b3, mean, std


def features(WL, WR, gamma=1.4):
    """Scale-free features of Riemann data (primitive rows [rho, u, p])."""
    WL = np.atleast_2d(np.asarray(WL, dtype=np.float64))
    WR = np.atleast_2d(np.asarray(WR, dtype=np.float64))
    rbar = 0.5 * (WL[:, 0] + WR[:, 0])
    pbar = 0.5 * (WL[:, 2] + WR[:, 2])
    cbar = np.sqrt(gamma * pbar / rbar)
    x = np.stack([np.log(WL[:, 0] / rbar), np.log(WR[:, 0] / rbar), np.log(WL[:, 2] / pbar),
                  np.log(WR[:, 2] / pbar), WL[:, 1] / cbar, WR[:, 1] / cbar], axis=1)
    return x, pbar


def forward(P, x):
    W1, b1, W2, b2, W3, b3, mean, std = unpack(P)
    z = (np.asarray(x, dtype=np.float64) - mean) / std
    h1 = np.tanh(z @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    return h2 @ W3 + b3


def backward(P, x, dy):
    """Gradient of sum_s dy_s y_s with respect to the 1313 weights, where y_s is
    the network output for sample s and dy_s the given upstream gradient."""
    W1, b1, W2, b2, W3, b3, mean, std = unpack(P)
    z = (np.asarray(x, dtype=np.float64) - mean) / std
    dy = np.asarray(dy, dtype=np.float64)
    h1 = np.tanh(z @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    d2 = np.outer(dy, W3) * (1 - h2 * h2)  # upstream gradient at pre-activation 2
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1 - h1 * h1)         # upstream gradient at pre-activation 1
    gW1 = d1.T @ z
    gb1 = d1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])


def loss(P, x, t):
    r = forward(P, x) - np.asarray(t, dtype=np.float64)
    return float(np.mean(r * r))


def loss_grad(P, x, t):
    """Gradient of the mean squared error with respect to the 1313 weights."""
    W1, b1, W2, b2, W3, b3, mean, std = unpack(P)
    n = x.shape[0]
    z = (np.asarray(x, dtype=np.float64) - mean) / std
    h1 = np.tanh(z @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ W3 + b3
    dy = 2.0 * (y - t) / n                # d loss / d y
    gW3 = h2.T @ dy
    gb3 = dy.sum()
    d2 = np.outer(dy, W3) * (1 - h2 * h2)  # d loss / d (pre-activation 2)
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (1 - h1 * h1)
    gW1 = d1.T @ z
    gb1 = d1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])


def adam(P, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of the weights (normaliser untouched); returns new (P, m, v)."""
    P = np.array(P, dtype=np.float64)
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    P[:NW] -= lr * mh / (np.sqrt(vh) + eps)
    return P, m, v
