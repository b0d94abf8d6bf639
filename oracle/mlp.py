"""Oracle: the warm-start perceptron in binary64 (forward, backward, Adam).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Network n_in -> H -> H -> n_out with tanh hidden layers and a linear output:
    H1 = tanh(X W1 + b1),  H2 = tanh(H1 W2 + b2),  Y = H2 W3 + b3
Loss: L = sum (Y - T)^2 / (batch * n_out).  Gradients by the chain rule written out layer by
layer; Adam as published by Kingma and Ba (bias-corrected moments).  Pinned against central
finite differences of L and against torch autograd on the CPU.
"""
from __future__ import annotations

import numpy as np


def init_params(n_in, n_hidden, n_out, seed=0):
    """LeCun-uniform initial weights U(-sqrt(3/fan_in), sqrt(3/fan_in)), zero biases."""
    rng = np.random.default_rng(seed)

    def w(fi, fo):
        a = np.sqrt(3.0 / fi)
        return rng.uniform(-a, a, (fi, fo))
    return dict(W1=w(n_in, n_hidden), b1=np.zeros(n_hidden), W2=w(n_hidden, n_hidden), b2=np.zeros(n_hidden),
                W3=w(n_hidden, n_out), b3=np.zeros(n_out))


def forward(P, X):
    H1 = np.tanh(X @ P["W1"] + P["b1"])
    H2 = np.tanh(H1 @ P["W2"] + P["b2"])
    Y = H2 @ P["W3"] + P["b3"]
    return H1, H2, Y


def loss(P, X, T):
    return float(np.sum((forward(P, X)[2] - T) ** 2) / T.size)


def backward(P, X, T):
    H1, H2, Y = forward(P, X)
    dY = 2.0 * (Y - T) / T.size
    G = {}
    G["W3"] = H2.T @ dY
    G["b3"] = dY.sum(axis=0)
    dZ2 = (dY @ P["W3"].T) * (1.0 - H2 * H2)
    G["W2"] = H1.T @ dZ2
    G["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["W2"].T) * (1.0 - H1 * H1)
    G["W1"] = X.T @ dZ1
    G["b1"] = dZ1.sum(axis=0)
    return float(np.sum((Y - T) ** 2) / T.size), G


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1**step)
    vhat = v / (1 - b2**step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
