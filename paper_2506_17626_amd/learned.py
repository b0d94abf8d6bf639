"""Learned warm start for the parametric 2D Poisson family: orchestration only.

Every computation runs in the HIP library (right-hand-side scaling, multi-RHS LSQR, target
standardisation, perceptron training and inference, decoding the starts, warm-started LSQR);
this module only draws the family's parameters and right-hand-side values (from
``instances``), moves them to the device and calls the C ABI in order.

Network input (one row per member of the family): [a_1..a_4, m_1/30..m_4/30, n_1/30..n_4/30];
target: the LSQR solution y (preconditioned coordinates), standardised per coordinate.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import instances as I
from . import rfm


def encode(params: np.ndarray, maxfreq: int) -> np.ndarray:
    nm = params.shape[1] // 3
    x = params.astype(np.float64).copy()
    x[:, nm:] /= maxfreq
    return x.astype(np.float32)


def family_rhs(inst, prob, params: np.ndarray):
    """Weighted right-hand sides [N, n] of the family members (device, binary64)."""
    rhs = I.poisson2d_family_rhs(inst, params)                     # [n, N] unscaled values
    dev = prob["weight"].device
    return rfm.rfm_weighted_rhs(prob["weight"], torch.from_numpy(np.ascontiguousarray(rhs.T)).to(dev))


@dataclass
class TrainingSet:
    X: torch.Tensor          # [n, 12] binary32 inputs
    T: torch.Tensor          # [n, ncols] binary32 targets (standardised after `standardize`)
    iters: np.ndarray        # LSQR iterations per member
    stops: np.ndarray


def solve_members(plan, fact, inst, prob, params, maxfreq, tol=1e-8, maxit=20000, group=64, progress=None):
    """Solve every member with multi-RHS LSQR; targets as binary32 rows.  ``progress`` (nullable)
    is called with (members done, members) after every group."""
    L = plan.layout
    dev = prob["weight"].device
    n = params.shape[0]
    T = torch.empty(n, L.ncols, dtype=torch.float32, device=dev)
    iters = np.zeros(n, dtype=np.int64)
    stops = np.zeros(n, dtype=np.int32)
    ws = None
    for g0 in range(0, n, group):
        chunk = params[g0:g0 + group]
        Hm = family_rhs(inst, prob, chunk)
        Y, it, sp = rfm.rfm_lsqr_multi(plan, fact, Hm, atol=tol, btol=tol, maxit=maxit, ws=ws)
        rfm.rfm_solutions_to_rows(Y, g0, T)
        iters[g0:g0 + len(chunk)] = it
        stops[g0:g0 + len(chunk)] = sp
        if progress is not None:
            progress(g0 + len(chunk), n)
    X = torch.from_numpy(encode(params, maxfreq)).to(dev)
    return TrainingSet(X, T, iters, stops)


def init_network(n_in, n_hidden, n_out, seed, device):
    """LeCun-uniform weights from the seeded generator, zero biases (binary32, device)."""
    rng = I.Rng(seed, stream=7)

    def w(fi, fo):
        a = np.sqrt(3.0 / fi)
        return torch.from_numpy(rng.uniform(-a, a, fi * fo).reshape(fi, fo).astype(np.float32)).to(device)
    z = lambda k: torch.zeros(k, dtype=torch.float32, device=device)
    return dict(W1=w(n_in, n_hidden), b1=z(n_hidden), W2=w(n_hidden, n_hidden), b2=z(n_hidden),
                W3=w(n_hidden, n_out), b3=z(n_out))


@dataclass
class WarmStartModel:
    P: dict
    mean: torch.Tensor
    sd: torch.Tensor
    maxfreq: int
    loss_history: np.ndarray

    def starts(self, plan, fact, params: np.ndarray):
        """LSQR starts [ncols, n] (binary64) for family members (a vector for one member)."""
        X = torch.from_numpy(encode(params, self.maxfreq)).to(self.mean.device)
        _, _, pred = rfm.rfm_mlp_forward(self.P, X)
        return rfm.rfm_decode_start(plan, fact, pred, self.mean, self.sd)


def train_warm_start(ts: TrainingSet, hidden=512, epochs=100, batch=256, lr=1e-3, seed=0, maxfreq=30):
    mean, sd = rfm.rfm_standardize_columns(ts.T)
    P = init_network(ts.X.shape[1], hidden, ts.T.shape[1], seed, ts.X.device)
    hist = rfm.rfm_mlp_train(P, ts.X, ts.T, epochs=epochs, batch=batch, lr=lr, seed=seed)
    return WarmStartModel(P, mean, sd, maxfreq, hist)
