"""Oracle: Algorithm 2 end to end, back-substitution, ansatz evaluation and error metric.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* coefficients: a_hat_j = R_hat_j^{-1} y_j by back-substitution, placed at the
  kept (dominant) columns; every other coefficient is exactly 0
  (Algorithm 2, output step).  Global column index of (j, k) is
  feat_off[j] + k (the paper's l = (j-1)K + k with per-subdomain K_j).
* u_hat(x) = sum_j w_j(x) sum_k a_jk phi_jk(x)                (eq. elm_solution)
* e_L1 = mean |u_hat - u| / std(u) over a regular test grid, std the
  population standard deviation of the true values (Section 4.2, performance
  evaluation).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import assembly, lsqr as lsqr_mod, rrqr


def back_substitute(R: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Solve R x = y for upper-triangular R, row by row from the bottom."""
    r = R.shape[0]
    x = np.zeros(r)
    for i in range(r - 1, -1, -1):
        x[i] = (y[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x


def coefficients(inst, facts, y: np.ndarray) -> np.ndarray:
    """Global coefficient vector a (length sum K_j), zeros at dropped columns."""
    a = np.zeros(int(inst.feat_off[-1]))
    yoff = lsqr_mod.rank_offsets([f.rank for f in facts])
    for j, f in enumerate(facts):
        if f.rank == 0:
            continue
        ahat = back_substitute(f.R, y[yoff[j]:yoff[j + 1]])
        a[inst.feat_off[j] + f.kept] = ahat
    return a


def evaluate(inst, a: np.ndarray, xt: np.ndarray) -> np.ndarray:
    """u_hat at points xt for coefficients a (eq. elm_solution), times the hard-constraint
    factor g when the instance has one (Section 5.1)."""
    N, d = xt.shape
    rows = [np.nonzero(assembly.support_mask(xt, inst.mu[j], inst.hw[j]))[0] for j in range(inst.J)]
    S = np.zeros(N)
    what = []
    for j in range(inst.J):
        W, _, _ = assembly.unnormalised_window(xt[rows[j]], inst.mu[j], inst.hw[j])
        S[rows[j]] += W
        what.append(W)
    u = np.zeros(N)
    for j in range(inst.J):
        r = rows[j]
        if r.size == 0:
            continue
        k0, k1 = inst.feat_off[j], inst.feat_off[j + 1]
        phi, _, _ = assembly.block_features(inst, j, xt[r])
        u[r] += (what[j] / S[r]) * (phi @ a[k0:k1])
    if inst.ansatz is not None:
        u = u * np.asarray(inst.ansatz(xt))[:, 0]   # u~ = g u_hat
    return u


def l1_error(inst, a: np.ndarray, npts: int | None = None) -> float:
    xt = inst.test_points(npts)
    uh = evaluate(inst, a, xt)
    ue = inst.exact(xt)
    return float(np.mean(np.abs(uh - ue)) / np.std(ue))


@dataclass
class Solution:
    rows: list
    blocks: list
    h: np.ndarray
    facts: list
    y: np.ndarray
    a: np.ndarray
    info: object


def solve(inst, tau=1e-12, form="q", atol=1e-8, btol=1e-8, maxit=20000, y0=None) -> Solution:
    """Algorithm 2: assemble, filter every block, LSQR on the preconditioned system,
    back-substitute and zero the dropped columns."""
    rows, blocks, h = assembly.assemble(inst)
    facts = rrqr.filter_blocks(blocks, tau)
    if form == "q":
        A = lsqr_mod.QForm(inst.N, rows, [f.Q for f in facts])
    else:
        A = lsqr_mod.RForm(inst.N, rows, [b[:, f.kept] for b, f in zip(blocks, facts)],
                           [f.R for f in facts])
    y, info = lsqr_mod.lsqr(A, h, y0=y0, atol=atol, btol=btol, maxit=maxit)
    a = coefficients(inst, facts, y)
    return Solution(rows, blocks, h, facts, y, a, info)
