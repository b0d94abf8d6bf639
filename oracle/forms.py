"""Oracle: the precision form (narrow operand + binary64 residual refinement).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The preconditioned operator of Proposition 3.1 is applied with Q_hat rounded to binary32
(round to nearest even) or to bfloat16 (the binary32 value rounded to nearest even on its
upper 16 bits), products and sums in binary32.  Refinement: residual and stopping test in
binary64 with the full operator, correction by LSQR on the narrow operator:

    y <- y0;  repeat:  r = h - A y;  stop by S1/S2 on the explicit r and A^T r;
                       d = LSQR(A_low, r; atol = btol = inner_tol);  y <- y + d
    until ||A^T r|| stops falling by at least half per step; then finish with binary64 LSQR
    on the full operator warm-started from y (the "polish").

Why the polish: the systems here keep a residual floor r* (they are least-squares, not
consistent), and refinement through a perturbed operator converges to A_low^T (h - A y) = 0
rather than A^T (h - A y) = 0, so ||A^T r|| / (||A|| ||r||) stalls near u_low.

Rounding, the narrow operator and the loop are written out here independently of the GPU
path; the pins check the rounding against torch's bfloat16 conversion and hand-worked ties,
and the refined solution against the dense binary64 least-squares solution.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lsqr as lsqr_mod


def round_f32(x: np.ndarray) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """bfloat16 values (returned as float32): binary32 rounding, then round to nearest even
    keeping the upper 16 bits."""
    f = round_f32(x)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32)


class NarrowQForm:
    """A_low = sum_j V_j^T round(Q_hat_j) W_hat_j with binary32 products and sums."""

    def __init__(self, N, rows, Qs, dtype="f32"):
        rnd = round_f32 if dtype == "f32" else round_bf16
        self.N = N
        self.rows = rows
        self.Qs = [rnd(Q) for Q in Qs]
        self.yoff = lsqr_mod.rank_offsets([Q.shape[1] for Q in Qs])
        self.n = int(self.yoff[-1])

    def matvec(self, y):
        out = np.zeros(self.N)
        for j, (r, Q) in enumerate(zip(self.rows, self.Qs)):
            out[r] += (Q @ y[self.yoff[j]:self.yoff[j + 1]].astype(np.float32)).astype(np.float64)
        return out

    def rmatvec(self, u):
        parts = [(Q.T @ u[r].astype(np.float32)).astype(np.float64) for r, Q in zip(self.rows, self.Qs)]
        return np.concatenate(parts) if parts else np.zeros(0)


@dataclass
class RefineInfo:
    outer: int = 0
    inner_iters: int = 0
    polish_iters: int = 0
    stop: int = 0
    history: list = None


def refine(A, A_low, h, y0=None, atol=1e-8, btol=1e-8, inner_tol=1e-4, max_outer=20,
           max_inner=100000, anorm=None, polish_maxit=100000):
    """Binary64 residual refinement around LSQR on the narrow operator, then a binary64
    polish when the explicit ||A^T r|| stops falling (or after max_outer steps).  The first
    step runs the narrow LSQR on h from the current y; later steps solve for a correction
    of the binary64 residual."""
    if anorm is None:
        anorm = float(np.sqrt(A.n))
    y = np.zeros(A.n) if y0 is None else np.array(y0, dtype=np.float64, copy=True)
    hn = float(np.linalg.norm(h))
    info = RefineInfo(history=[])
    prev_at = np.inf
    while True:
        r = h - A.matvec(y)
        rn = float(np.linalg.norm(r))
        at = float(np.linalg.norm(A.rmatvec(r)))
        yn = float(np.linalg.norm(y))
        info.history.append((rn, at))
        if rn == 0.0 or at == 0.0:
            info.stop = 4
            return y, info
        if rn <= btol * hn + atol * anorm * yn:
            info.stop = 1
            return y, info
        if at <= atol * anorm * rn:
            info.stop = 2
            return y, info
        if info.outer >= max_outer or at > 0.5 * prev_at:
            break
        prev_at = at
        if info.outer == 0:
            # first step: the narrow solve on h itself from the current y, so its rule is taken
            # relative to ||h|| and ||y|| (from y = 0 this is the correction solve on r = h)
            y, inner = lsqr_mod.lsqr(A_low, h, y0=y, atol=inner_tol, btol=inner_tol, maxit=max_inner,
                                     anorm=anorm)
        else:
            d, inner = lsqr_mod.lsqr(A_low, r, atol=inner_tol, btol=inner_tol, maxit=max_inner, anorm=anorm)
            y = y + d
        info.inner_iters += inner.iters
        info.outer += 1
    y, pol = lsqr_mod.lsqr(A, h, y0=y, atol=atol, btol=btol, maxit=polish_maxit, anorm=anorm)
    info.polish_iters = pol.iters
    info.stop = pol.stop
    return y, info
