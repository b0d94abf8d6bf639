"""Pins of the oracle's Golub-Kahan condition estimates against dense singular values."""
import numpy as np

from oracle import conditioning as cond


class Dense:
    def __init__(self, M):
        self.M = np.asarray(M, dtype=np.float64)
        self.n = self.M.shape[1]

    def matvec(self, x):
        return self.M @ x

    def rmatvec(self, y):
        return self.M.T @ y


def test_first_step_closed_forms():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((9, 5))
    h = rng.standard_normal(9)
    alpha, beta = cond.golub_kahan(Dense(M), h, 3)
    assert np.isclose(beta[0], np.linalg.norm(h), rtol=1e-15)
    assert np.isclose(alpha[0], np.linalg.norm(M.T @ h) / np.linalg.norm(h), rtol=1e-14)
    # beta_2 u_2 = A v_1 - alpha_1 u_1 with v_1 = A^T u_1 / alpha_1
    u1 = h / beta[0]
    v1 = M.T @ u1 / alpha[0]
    assert np.isclose(beta[1], np.linalg.norm(M @ v1 - alpha[0] * u1), rtol=1e-13)


def test_full_bidiagonalisation_reproduces_the_singular_values_of_a_diagonal_operator():
    """After n steps on an n x n operator the Ritz values are its singular values (a mild
    spectrum: without reorthogonalisation a wide one loses orthogonality within n steps and
    the smallest Ritz value lags, which the next test allows for)."""
    d = np.array([4.0, 3.0, 2.5, 2.0, 1.5, 1.0])
    h = np.ones(len(d))
    alpha, beta = cond.golub_kahan(Dense(np.diag(d)), h, len(d))
    smax, smin = cond.ritz_extremes(alpha, beta, len(d))
    assert np.isclose(smax, d.max(), rtol=1e-10)
    assert np.isclose(smin, d.min(), rtol=1e-10)
    assert beta[len(d)] < 1e-10 * beta[0]  # the Krylov space is complete


def test_ritz_extremes_lie_inside_the_spectrum_and_widen_with_k():
    """sigma_max(B_k) <= sigma_max(A), sigma_min(B_k) >= sigma_min(A), and their ratio never
    falls as k grows: a lower bound of kappa(A)."""
    rng = np.random.default_rng(1)
    U, _ = np.linalg.qr(rng.standard_normal((40, 15)))
    V, _ = np.linalg.qr(rng.standard_normal((15, 15)))
    s = np.logspace(0, -4, 15)
    M = U @ np.diag(s) @ V.T
    h = rng.standard_normal(40)
    alpha, beta = cond.golub_kahan(Dense(M), h, 15)
    prev = 1.0
    for k in range(1, 16):
        smax, smin = cond.ritz_extremes(alpha, beta, k)
        assert smax <= s[0] * (1 + 1e-12) and smin >= s[-1] * (1 - 1e-9)
        assert smax / smin >= prev * (1 - 1e-12)
        prev = smax / smin
    # the largest Ritz value converges within a few steps, the smallest lags (a lower bound)
    assert np.isclose(cond.ritz_extremes(alpha, beta, 6)[0], s[0], rtol=1e-8)
    assert 10.0 < prev <= s[0] / s[-1]


def test_bidiagonal_shape_and_entries():
    alpha = np.array([1.0, 2.0, 3.0, 4.0])
    beta = np.array([9.0, 5.0, 6.0, 7.0])
    B = cond.bidiagonal(alpha, beta, 3)
    assert B.shape == (4, 3)
    assert np.array_equal(np.diag(B), [1.0, 2.0, 3.0])
    assert np.array_equal(np.diag(B, -1), [5.0, 6.0, 7.0])
    assert np.count_nonzero(B) == 6


def test_m_form_is_the_block_sum_of_kept_columns():
    """The unpreconditioned operator: column (j, k) is the kept column of M_j on the rows of
    block j, and rmatvec is its adjoint."""
    from oracle import assembly, rrqr
    from oracle import lsqr as olsqr
    from paper_2506_17626_amd import instances as I

    inst = I.tiny("poisson2d")
    rows, blocks, h = assembly.assemble(inst)
    facts = rrqr.filter_blocks(blocks, 1e-8)
    A = olsqr.MForm(inst.N, rows, [b[:, f.kept] for b, f in zip(blocks, facts)])
    off = np.concatenate([[0], np.cumsum([f.rank for f in facts])])
    j = int(np.argmax([f.rank for f in facts]))
    k = facts[j].rank // 2
    e = np.zeros(A.n)
    e[off[j] + k] = 1.0
    col = np.zeros(inst.N)
    col[rows[j]] = blocks[j][:, facts[j].kept[k]]
    assert np.array_equal(A.matvec(e), col)
    rng = np.random.default_rng(2)
    x, u = rng.standard_normal(A.n), rng.standard_normal(inst.N)
    assert np.isclose(A.matvec(x) @ u, x @ A.rmatvec(u), rtol=1e-12)
