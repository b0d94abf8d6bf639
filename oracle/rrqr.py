"""Oracle: sigma-RRQR filtering of one block (Algorithm 1, Section 2.3 definition).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper asks for a factorisation M_j Pi_j = Q_j [R_j *; 0 T_j] whose trailing
part is small, keeps the columns of R_j, and measures the threshold sigma
relative to the leading diagonal entry of R_j (Algorithm 1 and the note after
it).  It names strong RRQR as one way to get such a factorisation; this oracle
uses the classical Businger-Golub column-pivoted Householder QR:

  at step s pick, among the columns not yet chosen, the one whose component
  orthogonal to the span of the chosen columns is largest (ties between
  bit-equal norms go to the smallest original feature id); stop at the first
  step whose largest such component |R_ss| is <= tau * |R_00|; the kept set is
  the r = s columns chosen before.

Norms are recomputed from scratch at every step (no downdating).  The
Householder reflector of column s is the LAPACK-style one: beta =
-sign(alpha) ||x||, v = [1, x_2:/(alpha - beta)], tau_h = (beta - alpha)/beta.
After the loop the kept factor is sign-normalised so diag(R_hat) > 0 (row k
of R_hat and column k of Q_hat flipped together), which leaves Q_hat R_hat
unchanged.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class RRQRResult:
    rank: int
    kept: np.ndarray        # [rank] local feature ids in pivot order
    perm: np.ndarray        # [n] full pivot order reached (entries >= steps taken are untouched)
    R: np.ndarray           # [rank, rank] upper triangular, positive diagonal
    Q: np.ndarray           # [m, rank] orthonormal columns
    ratios: np.ndarray      # |R_ss| / |R_00| for every step taken (incl. the stopping step)
    gaps: np.ndarray        # (best - runner-up) / |R_00| of the pivot choice at each step


def qrcp_filter(Mj: np.ndarray, tau: float) -> RRQRResult:
    A = np.array(Mj, dtype=np.float64, copy=True)
    m, n = A.shape
    perm = np.arange(n)
    taus = []
    ratios, gaps = [], []
    ref = 0.0
    r = min(m, n)
    for s in range(min(m, n)):
        c = np.sqrt(np.sum(A[s:, s:] * A[s:, s:], axis=0))       # exact trailing norms
        best = c.max()
        ties = np.nonzero(c == best)[0]
        p = s + ties[np.argmin(perm[s + ties])]                   # tie -> smallest feature id
        if s == 0:
            ref = best
            if ref == 0.0:
                r = 0
                break
        ratios.append(best / ref)
        if c.size > 1:
            second = np.partition(c, -2)[-2] if ties.size == 1 else best
            gaps.append((best - second) / ref)
        else:
            gaps.append(np.inf)
        if best <= tau * ref:
            r = s
            break
        if p != s:
            A[:, [s, p]] = A[:, [p, s]]
            perm[[s, p]] = perm[[p, s]]
        alpha = A[s, s]
        sig2 = np.sum(A[s + 1:, s] ** 2)
        if sig2 == 0.0:
            th = 0.0
            v = np.zeros(m - s)
            v[0] = 1.0
        else:
            beta = -np.copysign(np.sqrt(alpha * alpha + sig2), alpha if alpha != 0 else 1.0)
            v = np.concatenate([[1.0], A[s + 1:, s] / (alpha - beta)])
            th = (beta - alpha) / beta
            A[s, s] = beta
            A[s + 1:, s] = v[1:]
        taus.append((th, v))
        if s + 1 < n:
            F = v @ A[s:, s + 1:]
            A[s:, s + 1:] -= th * np.outer(v, F)
    R = np.triu(A[:r, :r]).copy()
    # explicit Q_hat = H_0 ... H_{r-1} [I_r; 0]
    Q = np.zeros((m, r))
    Q[:r, :r] = np.eye(r)
    for s in range(r - 1, -1, -1):
        th, v = taus[s]
        Q[s:, :] -= th * np.outer(v, v @ Q[s:, :])
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    R = sgn[:, None] * R
    Q = Q * sgn[None, :]
    return RRQRResult(r, perm[:r].copy(), perm, R, Q, np.array(ratios), np.array(gaps))


def filter_blocks(blocks, tau: float):
    """Algorithm 1: the sigma-RRQR filter applied independently to every block."""
    return [qrcp_filter(Mj, tau) for Mj in blocks]


# ---------------------------------------------------------------- strong RRQR
# Gu and Eisenstat (1996): for a fixed rank r, with R = [A B; 0 C] the triangular factor of
# M_j in pivot order, the factorisation is strong with parameter f > 1 when every
#   rho_iq = (A^-1 B)_iq^2 + (gamma_q / omega_i)^2 <= f^2,
# gamma_q = ||C e_q|| (the trailing column norms) and 1/omega_i = ||e_i^T A^-1|| (the row norms
# of A^-1).  While it is not, exchanging kept column i for trailing column q at the largest
# rho multiplies |det A| by sqrt(rho) > f, so the exchanges end.  The rank is the
# sigma-filter's (Section 2.3 names strong RRQR as one admissible rank-revealing QR).

def strong_measure(Mj: np.ndarray, perm: np.ndarray, r: int):
    """rho [r, n-r] of the pivot order perm at rank r, from a fresh QR of the permuted block."""
    m, n = Mj.shape
    Rf = np.linalg.qr(np.asarray(Mj, dtype=np.float64)[:, perm], mode="r")   # [min(m,n), n]
    A, B, C = Rf[:r, :r], Rf[:r, r:], Rf[r:, r:]
    Ainv = np.linalg.solve(A, np.eye(r))
    W = Ainv @ B
    gam2 = np.sum(C * C, axis=0) if C.shape[0] else np.zeros(n - r)
    om2 = np.sum(Ainv * Ainv, axis=1)
    return W * W + gam2[None, :] * om2[:, None]


def _argmax_first(rho: np.ndarray):
    """Position of the largest entry, ties to the smaller row, then column."""
    best = rho.max()
    i, q = np.argwhere(rho == best)[0]
    return int(i), int(q), float(best)


def strong_filter(Mj: np.ndarray, tau: float, f: float = 2.0, max_rounds: int = 32):
    """The sigma-filter's rank with Gu-Eisenstat exchanges; returns (RRQRResult of the final
    order, swaps, largest rho of the last test)."""
    base = qrcp_filter(Mj, tau)
    m, n = np.asarray(Mj).shape
    r, perm = base.rank, base.perm.copy()
    swaps, last = 0, 0.0
    for _ in range(max_rounds):
        if r == 0 or r >= n:
            last = 0.0
            break
        rho = strong_measure(Mj, perm, r)
        i, q, last = _argmax_first(rho)
        if last <= f * f:
            break
        perm[[i, r + q]] = perm[[r + q, i]]
        swaps += 1
    if swaps == 0:
        return base, 0, last
    Qf, Rf = np.linalg.qr(np.asarray(Mj, dtype=np.float64)[:, perm[:r]])
    sgn = np.where(np.diag(Rf) < 0, -1.0, 1.0)
    res = RRQRResult(r, perm[:r].copy(), perm, sgn[:, None] * Rf, Qf * sgn[None, :],
                     np.array([]), np.array([]))
    return res, swaps, last
