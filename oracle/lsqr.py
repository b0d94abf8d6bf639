"""Oracle: the right-preconditioned operator and LSQR (Algorithm 2, Proposition 3.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Operator.  With the filtered blocks M_hat_j = Q_hat_j R_hat_j the preconditioned
matrix is M_hat S^{-1} = sum_j V_j^T M_hat_j R_hat_j^{-1} W_hat_j, which equals
sum_j V_j^T Q_hat_j W_hat_j (Proposition 3.1).  Both realisations are given:
``QForm`` applies the explicit orthonormal factors, ``RForm`` applies the
kept columns of M_j after a triangular solve with R_hat_j (the preconditioner
S^{-1} is never formed, only back-substitution is used).  Rows shared by
several subdomains are summed in ascending subdomain order.

Unknowns y are stored compactly: block j owns y[yoff[j] : yoff[j] + r_j] in
pivot order.

LSQR.  Golub-Kahan bidiagonalisation with the Givens-rotation update of
Paige and Saunders (1982), started from y0 (r0 = h - A y0).  Stopping rule:
with a fixed operator norm estimate ||A|| = ||A||_F = sqrt(sum_j r_j) (exact for
the Q form, whose columns have unit norm), stop when
  (S1) ||r|| <= btol ||h|| + atol ||A|| ||y||      or
  (S2) ||A^T r|| <= atol ||A|| ||r||,
using the recurrence estimates ||r|| ~ phibar_{i+1} and
||A^T r|| ~ phibar_{i+1} alpha_{i+1} |c_i|; or on breakdown (alpha or beta = 0,
exact solution) or at maxit.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.linalg import solve_triangular


def rank_offsets(ranks):
    return np.concatenate([[0], np.cumsum(ranks)]).astype(np.int64)


class QForm:
    """A = sum_j V_j^T Q_hat_j W_hat_j (Proposition 3.1)."""

    def __init__(self, N, rows, Qs):
        self.N = N
        self.rows = rows
        self.Qs = Qs
        self.yoff = rank_offsets([Q.shape[1] for Q in Qs])
        self.n = int(self.yoff[-1])

    def matvec(self, y):
        out = np.zeros(self.N)
        for j, (r, Q) in enumerate(zip(self.rows, self.Qs)):
            out[r] += Q @ y[self.yoff[j]:self.yoff[j + 1]]
        return out

    def rmatvec(self, u):
        return np.concatenate([Q.T @ u[r] for r, Q in zip(self.rows, self.Qs)]) if self.Qs else np.zeros(0)


class MForm(QForm):
    """A = M_hat = sum_j V_j^T M_hat_j W_hat_j, the kept columns of M_j without the
    preconditioner: the same block sum as the Q form with M_hat_j in place of Q_hat_j (for
    condition estimates of the unpreconditioned system)."""


class RForm:
    """A = M_hat S^{-1}, S^{-1} applied block by block by back-substitution with R_hat_j."""

    def __init__(self, N, rows, Mhats, Rs):
        self.N = N
        self.rows = rows
        self.Mhats = Mhats
        self.Rs = Rs
        self.yoff = rank_offsets([R.shape[0] for R in Rs])
        self.n = int(self.yoff[-1])

    def matvec(self, y):
        out = np.zeros(self.N)
        for j, (r, M, R) in enumerate(zip(self.rows, self.Mhats, self.Rs)):
            yj = y[self.yoff[j]:self.yoff[j + 1]]
            if yj.size:
                out[r] += M @ solve_triangular(R, yj, lower=False)
        return out

    def rmatvec(self, u):
        parts = []
        for r, M, R in zip(self.rows, self.Mhats, self.Rs):
            if R.shape[0]:
                parts.append(solve_triangular(R, M.T @ u[r], lower=False, trans="T"))
            else:
                parts.append(np.zeros(0))
        return np.concatenate(parts) if parts else np.zeros(0)


@dataclass
class LSQRInfo:
    iters: int = 0
    stop: int = 0            # 1 = S1, 2 = S2, 3 = maxit, 4 = breakdown (exact solution)
    rnorm_est: float = 0.0
    artnorm_est: float = 0.0
    history: list = field(default_factory=list)


def lsqr(A, h, y0=None, atol=1e-8, btol=1e-8, maxit=10000, anorm=None, keep_history=False):
    """LSQR for min ||A y - h||, returning (y, LSQRInfo)."""
    n = A.n
    if anorm is None:
        anorm = float(np.sqrt(n))
    hnorm = float(np.linalg.norm(h))
    y = np.zeros(n) if y0 is None else np.array(y0, dtype=np.float64, copy=True)
    info = LSQRInfo()
    u = h - A.matvec(y) if y0 is not None else np.array(h, dtype=np.float64, copy=True)
    beta = float(np.linalg.norm(u))
    if beta == 0.0:
        info.stop = 4
        return y, info
    u = u / beta
    v = A.rmatvec(u)
    alpha = float(np.linalg.norm(v))
    if alpha == 0.0:
        info.stop = 4
        info.rnorm_est = beta
        return y, info
    v = v / alpha
    w = v.copy()
    phibar, rhobar = beta, alpha
    for it in range(1, maxit + 1):
        p = A.matvec(v) - alpha * u
        beta = float(np.linalg.norm(p))
        if beta > 0.0:
            u = p / beta
            q = A.rmatvec(u) - beta * v
            alpha = float(np.linalg.norm(q))
            if alpha > 0.0:
                v = q / alpha
        else:
            alpha = 0.0
        rho = float(np.hypot(rhobar, beta))
        c = rhobar / rho
        s = beta / rho
        theta = s * alpha
        rhobar = -c * alpha
        phi = c * phibar
        phibar = s * phibar
        y = y + (phi / rho) * w
        w = v - (theta / rho) * w
        rnorm = phibar
        artnorm = phibar * alpha * abs(c)
        info.iters = it
        info.rnorm_est = rnorm
        info.artnorm_est = artnorm
        if keep_history:
            info.history.append((rnorm, artnorm))
        if beta == 0.0 or alpha == 0.0:
            info.stop = 4
            break
        ynorm = float(np.linalg.norm(y))
        if rnorm <= btol * hnorm + atol * anorm * ynorm:
            info.stop = 1
            break
        if artnorm <= atol * anorm * rnorm:
            info.stop = 2
            break
    else:
        info.stop = 3
    return y, info


def explicit_residuals(A, h, y, anorm=None):
    """Relative residual ||h - A y|| / ||h|| and eta = ||A^T r|| / (||A|| ||r||), recomputed."""
    if anorm is None:
        anorm = float(np.sqrt(A.n))
    r = h - A.matvec(y)
    rn = float(np.linalg.norm(r))
    at = float(np.linalg.norm(A.rmatvec(r)))
    return rn / float(np.linalg.norm(h)), (at / (anorm * rn) if rn > 0 else 0.0)
