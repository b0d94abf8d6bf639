"""Pins of the oracle perceptron: gradients against central finite differences and against
torch autograd (CPU, float64); Adam against its closed form on a quadratic."""
import numpy as np
import torch

from oracle import mlp


def _problem(seed=0):
    rng = np.random.default_rng(seed)
    P = mlp.init_params(5, 7, 3, seed)
    for k in ("b1", "b2", "b3"):
        P[k] = rng.standard_normal(P[k].shape) * 0.1
    X = rng.standard_normal((6, 5))
    T = rng.standard_normal((6, 3))
    return P, X, T


def test_gradients_match_central_differences():
    P, X, T = _problem()
    L, G = mlp.backward(P, X, T)
    assert abs(L - mlp.loss(P, X, T)) < 1e-15
    e = 1e-6
    for k in P:
        it = np.nditer(P[k], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            Pp = {kk: vv.copy() for kk, vv in P.items()}
            Pm = {kk: vv.copy() for kk, vv in P.items()}
            Pp[k][idx] += e
            Pm[k][idx] -= e
            fd = (mlp.loss(Pp, X, T) - mlp.loss(Pm, X, T)) / (2 * e)
            assert abs(fd - G[k][idx]) <= 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_gradients_match_torch_autograd():
    P, X, T = _problem(3)
    _, G = mlp.backward(P, X, T)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in P.items()}
    Xt, Tt = torch.tensor(X), torch.tensor(T)
    H1 = torch.tanh(Xt @ tp["W1"] + tp["b1"])
    H2 = torch.tanh(H1 @ tp["W2"] + tp["b2"])
    Y = H2 @ tp["W3"] + tp["b3"]
    L = ((Y - Tt) ** 2).sum() / Tt.numel()
    L.backward()
    for k in P:
        assert np.allclose(tp[k].grad.numpy(), G[k], rtol=1e-12, atol=1e-15), k


def test_adam_matches_closed_form_first_step_and_decreases_quadratic():
    # first step: m_hat = g, v_hat = g^2 -> p - lr * g / (|g| + eps)
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.1)
    assert np.allclose(p1, p - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    # a quadratic is driven towards its minimum
    p = np.array([3.0, -1.0])
    m = v = np.zeros(2)
    for s in range(1, 2001):
        p, m, v = mlp.adam_step(p, 2 * p, m, v, s, lr=1e-2)
    assert np.all(np.abs(p) < 1e-2)
