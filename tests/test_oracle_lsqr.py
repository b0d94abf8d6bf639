"""Pins of the oracle's preconditioned operator, LSQR and Algorithm 2 output.

Independent checks: the dense least-squares solution (numpy lstsq) of the
assembled preconditioned matrix, brute-force Krylov minimisers for the first
iterates, one-step termination for orthonormal columns, Proposition 3.1
(Q form = R form up to the rounding bound), the exact two-block condition
number of the remark after Theorem 3.2, the bound of Theorem 3.2, triangular
solves against scipy, and the manufactured-solution error of a full solve.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import assembly, lsqr, rrqr, solve
from paper_2506_17626_amd import instances as I


def _factored(inst, tau):
    rows, blocks, h = assembly.assemble(inst)
    facts = rrqr.filter_blocks(blocks, tau)
    return rows, blocks, h, facts


def _dense(A):
    return np.stack([A.matvec(e) for e in np.eye(A.n)], axis=1)


def test_operator_transpose_consistency():
    inst = I.tiny("poisson2d")
    rows, blocks, h, facts = _factored(inst, 1e-10)
    for A in (lsqr.QForm(inst.N, rows, [f.Q for f in facts]),
              lsqr.RForm(inst.N, rows, [b[:, f.kept] for b, f in zip(blocks, facts)], [f.R for f in facts])):
        rng = np.random.default_rng(0)
        x, u = rng.standard_normal(A.n), rng.standard_normal(inst.N)
        assert abs(u @ A.matvec(x) - A.rmatvec(u) @ x) < 1e-10 * np.linalg.norm(u) * np.linalg.norm(x) * 1e3


def test_proposition_3_1_q_form_equals_r_form():
    inst = I.tiny("poisson1d")
    rows, blocks, h, facts = _factored(inst, 1e-8)
    Aq = lsqr.QForm(inst.N, rows, [f.Q for f in facts])
    Ar = lsqr.RForm(inst.N, rows, [b[:, f.kept] for b, f in zip(blocks, facts)], [f.R for f in facts])
    rng = np.random.default_rng(1)
    for _ in range(3):
        x = rng.standard_normal(Aq.n)
        # a posteriori bound: c u ||M_hat|| ||R^{-1} x||
        bound = 0.0
        for j, (b, f) in enumerate(zip(blocks, facts)):
            xj = x[Aq.yoff[j]:Aq.yoff[j + 1]]
            bound += np.linalg.norm(b[:, f.kept], 2) * np.linalg.norm(scipy.linalg.solve_triangular(f.R, xj))
        diff = np.linalg.norm(Aq.matvec(x) - Ar.matvec(x))
        assert diff <= 100 * np.finfo(float).eps * bound
        assert diff <= 1e-5 * np.linalg.norm(x)


@pytest.mark.parametrize("name", ["poisson1d", "heat3d"])
def test_converged_lsqr_equals_dense_least_squares(name):
    inst = I.tiny(name)
    rows, blocks, h, facts = _factored(inst, 1e-8)
    A = lsqr.QForm(inst.N, rows, [f.Q for f in facts])
    y, info = lsqr.lsqr(A, h, atol=1e-14, btol=1e-14, maxit=5000)
    D = _dense(A)
    ystar = np.linalg.lstsq(D, h, rcond=None)[0]
    cond = np.linalg.cond(D)
    assert np.linalg.norm(y - ystar) <= 1e-12 * cond * np.linalg.norm(ystar)
    rel, eta = lsqr.explicit_residuals(A, h, y)
    assert eta < 1e-10


def test_first_iterates_are_krylov_minimisers():
    inst = I.tiny("poisson2d")
    rows, blocks, h, facts = _factored(inst, 1e-8)
    A = lsqr.QForm(inst.N, rows, [f.Q for f in facts])
    D = _dense(A)
    for k in range(1, 7):
        yk, info = lsqr.lsqr(A, h, atol=0.0, btol=0.0, maxit=k)
        assert info.iters == k
        # brute force: minimise ||D y - h|| over span{D^T h, (D^T D) D^T h, ...}
        basis = []
        vec = D.T @ h
        for _ in range(k):
            for b in basis:
                vec = vec - (b @ vec) * b
            for b in basis:
                vec = vec - (b @ vec) * b
            vec = vec / np.linalg.norm(vec)
            basis.append(vec)
            vec = D.T @ (D @ vec)
        B = np.stack(basis, 1)
        c = np.linalg.lstsq(D @ B, h, rcond=None)[0]
        ybf = B @ c
        assert np.linalg.norm(yk - ybf) <= 1e-9 * np.linalg.norm(ybf)


def test_orthonormal_operator_terminates_after_one_iteration():
    # one subdomain: the preconditioned operator has orthonormal columns, so LSQR
    # reaches the least-squares solution Q^T h in its first iteration
    inst = I.poisson1d(S=1, K=20, n=60, rho=0.3)
    rows, blocks, h, facts = _factored(inst, 1e-10)
    A = lsqr.QForm(inst.N, rows, [f.Q for f in facts])
    y, info = lsqr.lsqr(A, h, atol=1e-10, btol=1e-10)
    assert info.iters == 1 and info.stop in (2, 4)
    assert np.allclose(y, facts[0].Q.T @ h[rows[0]], rtol=1e-12, atol=1e-14)


def _overlap_coupling(rows, facts, j):
    common, ia, ib = np.intersect1d(rows[j], rows[j + 1], return_indices=True)
    return facts[j].Q[ia].T @ facts[j + 1].Q[ib]


def test_two_block_condition_number_closed_form():
    inst = I.poisson1d(S=2, K=12, n=40, rho=0.4)
    rows, blocks, h, facts = _factored(inst, 1e-8)
    A = lsqr.QForm(inst.N, rows, [f.Q for f in facts])
    a1 = np.linalg.norm(_overlap_coupling(rows, facts, 0), 2)
    assert a1 < 1
    kappa = np.linalg.cond(_dense(A))
    assert kappa == pytest.approx(np.sqrt((1 + a1) / (1 - a1)), rel=1e-10)


def test_theorem_3_2_bound_on_strip_blocks():
    """Theorem 3.2 on a chain of J blocks with orthonormal columns whose consecutive
    row sets overlap; the coupling is made weak by giving the overlap rows little weight
    before orthonormalising."""
    rng = np.random.default_rng(8)
    J, K, interior, ell = 7, 6, 25, 5
    rows, Qs = [], []
    start = 0
    for j in range(J):
        m = interior + (ell if j > 0 else 0) + (ell if j < J - 1 else 0)
        G = rng.standard_normal((m, K))
        lo = ell if j > 0 else 0
        hi = m - (ell if j < J - 1 else 0)
        G[:lo] *= 0.3
        G[hi:] *= 0.3
        Q, _ = np.linalg.qr(G)
        rows.append(np.arange(start, start + m))
        Qs.append(Q)
        start += m - ell
    N = start + ell
    A = lsqr.QForm(N, rows, Qs)
    couplings = []
    for j in range(J - 1):
        common, ia, ib = np.intersect1d(rows[j], rows[j + 1], return_indices=True)
        couplings.append(np.linalg.norm(Qs[j][ia].T @ Qs[j + 1][ib], 2))
    alpha = max(couplings)
    assert 2 * alpha < 1
    kappa = np.linalg.cond(_dense(A))
    assert kappa <= np.sqrt((1 + 2 * alpha) / (1 - 2 * alpha)) * (1 + 1e-12)
    # and the preconditioned operator of a real 1D feature problem is near the
    # strong-coupling end (alpha close to 1), where the bound does not apply
    inst = I.poisson1d(S=4, K=10, n=30, rho=0.2)
    rws, blocks, h, facts = _factored(inst, 1e-4)
    assert max(np.linalg.norm(_overlap_coupling(rws, facts, j), 2) for j in range(3)) > 0.5


def test_back_substitution_and_zero_columns():
    rng = np.random.default_rng(4)
    R = np.triu(rng.standard_normal((30, 30))) + 5 * np.eye(30)
    y = rng.standard_normal(30)
    assert np.allclose(solve.back_substitute(R, y), scipy.linalg.solve_triangular(R, y), rtol=1e-13)
    inst = I.tiny("poisson1d")
    sol = solve.solve(inst, tau=1e-8)
    kept_mask = np.zeros(int(inst.feat_off[-1]), bool)
    for j, f in enumerate(sol.facts):
        kept_mask[inst.feat_off[j] + f.kept] = True
    assert np.all(sol.a[~kept_mask] == 0.0)
    # M a reproduces the preconditioned residual: M a = M_hat S^{-1} y
    M = assembly.global_dense(inst, sol.rows, sol.blocks)
    A = lsqr.QForm(inst.N, sol.rows, [f.Q for f in sol.facts])
    assert np.linalg.norm(M @ sol.a - A.matvec(sol.y)) <= 1e-6 * np.linalg.norm(sol.h)


def test_manufactured_solution_error_1d_full_size():
    inst = I.workload("poisson1d")
    sol = solve.solve(inst, tau=1e-12, atol=1e-8, btol=1e-8)
    assert sol.info.stop in (1, 2)
    e = solve.l1_error(inst, sol.a)
    assert e < 1e-4
    # the filter drops most of the smooth, redundant features of this workload
    kept = sum(f.rank for f in sol.facts)
    assert 0.2 * 1280 < kept < 0.4 * 1280
