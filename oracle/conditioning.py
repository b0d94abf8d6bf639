"""Oracle: condition estimates of the least-squares operators from the Golub-Kahan
bidiagonalisation (Golub and Kahan 1965), the process LSQR runs (Paige and Saunders 1982).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Started from h, the lower bidiagonalisation builds orthonormal U_{k+1}, V_k and the
(k+1) x k lower bidiagonal B_k with A V_k = U_{k+1} B_k:
  beta_1 u_1 = h,            alpha_1 v_1 = A^T u_1,
  beta_{i+1} u_{i+1} = A v_i - alpha_i u_i,
  alpha_{i+1} v_{i+1} = A^T u_{i+1} - beta_{i+1} v_i,
with every alpha, beta >= 0 chosen to normalise.  B_k has alpha_1..alpha_k on its
diagonal and beta_2..beta_{k+1} below it.  Its singular values are Ritz values of A (in exact
arithmetic they interlace A's and reach them at k = rank), so sigma_max(B_k) and
sigma_min(B_k) approach sigma_max(A) and sigma_min(A) from inside, and their ratio is a
lower bound of kappa(A) that grows with k.  No reorthogonalisation, as in LSQR.
"""
import numpy as np


def golub_kahan(A, h, k):
    """k steps from h: arrays alpha[0..k] = alpha_1..alpha_{k+1} and beta[0..k] =
    beta_1..beta_{k+1} (a breakdown leaves the remaining entries 0)."""
    alpha = np.zeros(k + 1)
    beta = np.zeros(k + 1)
    beta[0] = float(np.linalg.norm(h))
    if beta[0] == 0.0:
        return alpha, beta
    u = np.asarray(h, dtype=np.float64) / beta[0]
    v = A.rmatvec(u)
    alpha[0] = float(np.linalg.norm(v))
    if alpha[0] == 0.0:
        return alpha, beta
    v = v / alpha[0]
    for i in range(k):
        p = A.matvec(v) - alpha[i] * u
        beta[i + 1] = float(np.linalg.norm(p))
        if beta[i + 1] == 0.0:
            break
        u = p / beta[i + 1]
        q = A.rmatvec(u) - beta[i + 1] * v
        alpha[i + 1] = float(np.linalg.norm(q))
        if alpha[i + 1] == 0.0:
            break
        v = q / alpha[i + 1]
    return alpha, beta


def bidiagonal(alpha, beta, k):
    """B_k, (k+1) x k, from the scalars of golub_kahan (or of an LSQR run)."""
    B = np.zeros((k + 1, k))
    for i in range(k):
        B[i, i] = alpha[i]
        B[i + 1, i] = beta[i + 1]
    return B


def ritz_extremes(alpha, beta, k):
    """(sigma_max, sigma_min) of B_k: the bidiagonalisation's estimates of A's extreme
    singular values after k steps."""
    s = np.linalg.svd(bidiagonal(alpha, beta, k), compute_uv=False)
    return float(s[0]), float(s[-1])
