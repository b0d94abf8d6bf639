"""Pins of the oracle's sigma-RRQR filter (Algorithm 1 with column-pivoted Householder QR).

Independent checks: reconstruction and orthogonality, the pivoting invariant
|R_{k+1,k+1}| <= |R_kk|, exact ranks on matrices built with a known spectral gap
(SVD by numpy as the definition of numerical rank), LAPACK's pivoted QR
(scipy dgeqp3) on generic matrices, duplicated columns, exact power-of-two
scaling, wide and zero blocks, and real feature blocks bracketed by SVD ranks.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import assembly, rrqr
from paper_2506_17626_amd import instances as I


def _check_factor(M, f, tol=1e-12):
    m, n = M.shape
    Mh = M[:, f.kept]
    assert np.linalg.norm(Mh - f.Q @ f.R) <= tol * max(np.linalg.norm(M), 1e-300)
    assert np.linalg.norm(f.Q.T @ f.Q - np.eye(f.rank)) <= tol * max(1, f.rank)
    d = np.diag(f.R)
    assert np.all(d > 0)
    assert np.all(np.triu(f.R) == f.R)
    slack = 10 * np.sqrt(m) * np.finfo(float).eps * (d[0] if f.rank else 0)
    assert np.all(d[1:] <= d[:-1] + slack)


@pytest.mark.parametrize("shape", [(40, 12), (97, 33), (12, 12), (9, 25)])
def test_full_rank_reconstruction_and_invariants(shape):
    rng = np.random.default_rng(sum(shape))
    M = rng.standard_normal(shape)
    f = rrqr.qrcp_filter(M, 0.0)
    assert f.rank == min(shape)
    _check_factor(M, f)
    assert sorted(f.perm) == list(range(shape[1]))


def test_pivots_match_lapack_on_generic_matrices():
    rng = np.random.default_rng(11)
    for trial in range(5):
        M = rng.standard_normal((60, 25)) * rng.uniform(0.5, 2.0, 25)
        f = rrqr.qrcp_filter(M, 0.0)
        _, R, piv = scipy.linalg.qr(M, mode="economic", pivoting=True)
        assert np.array_equal(f.kept, piv)
        assert np.allclose(np.abs(np.diag(R)), np.diag(f.R), rtol=1e-12)
        assert np.allclose(np.abs(R), np.abs(f.R), atol=1e-12 * np.abs(R).max())


@pytest.mark.parametrize("true_rank,tau", [(7, 1e-8), (15, 1e-12), (1, 1e-6), (20, 1e-12)])
def test_rank_equals_svd_rank_with_spectral_gap(true_rank, tau):
    rng = np.random.default_rng(true_rank)
    m, n = 70, 20
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.concatenate([np.logspace(0, -2, true_rank), np.full(n - true_rank, tau * 1e-5)])[:n]
    M = (U * s) @ V.T
    f = rrqr.qrcp_filter(M, tau)
    sv = np.linalg.svd(M, compute_uv=False)
    assert f.rank == true_rank == int(np.sum(sv > tau * sv[0] * 1e2))
    _check_factor(M, f)


def test_duplicated_columns_keep_one_copy_lowest_id():
    rng = np.random.default_rng(5)
    M = rng.standard_normal((50, 20))
    M[:, 12] = M[:, 4]
    M[:, 17] = M[:, 4]
    f = rrqr.qrcp_filter(M, 1e-12)
    assert f.rank == 18
    assert 4 in f.kept and 12 not in f.kept and 17 not in f.kept


def test_power_of_two_scaling_is_exact():
    rng = np.random.default_rng(9)
    M = rng.standard_normal((45, 30)) @ np.diag(np.logspace(0, -14, 30))
    f1 = rrqr.qrcp_filter(M, 1e-10)
    f2 = rrqr.qrcp_filter(M * 2.0**37, 1e-10)
    assert np.array_equal(f1.kept, f2.kept)
    assert np.array_equal(f1.R * 2.0**37, f2.R)
    assert np.array_equal(f1.Q, f2.Q)


def test_zero_and_wide_blocks():
    f = rrqr.qrcp_filter(np.zeros((10, 4)), 1e-12)
    assert f.rank == 0 and f.kept.size == 0 and f.Q.shape == (10, 0)
    rng = np.random.default_rng(2)
    M = rng.standard_normal((6, 15))
    f = rrqr.qrcp_filter(M, 1e-12)
    assert f.rank == 6
    _check_factor(M, f)


def test_threshold_is_relative_to_leading_diagonal():
    # columns with norms 1, 1e-3, 1e-6 (orthogonal): tau=1e-4 keeps two, tau=1e-7 keeps three
    M = np.zeros((5, 3))
    M[0, 0], M[1, 1], M[2, 2] = 1e-6, 1.0, 1e-3
    assert list(rrqr.qrcp_filter(M, 1e-4).kept) == [1, 2]
    assert list(rrqr.qrcp_filter(M, 1e-7).kept) == [1, 2, 0]
    # keep iff |R_ss| > tau |R_00|: a column exactly at the threshold is dropped
    assert rrqr.qrcp_filter(M, 1e-3).rank == 1
    assert rrqr.qrcp_filter(M * 7.0, 1e-4).rank == 2


@pytest.mark.parametrize("name", ["poisson1d", "poisson2d", "helmholtz2d_uneven"])
@pytest.mark.parametrize("tau", [1e-12, 1e-8])
def test_feature_blocks_rank_bracketed_by_svd(name, tau):
    inst = I.tiny(name)
    rows, blocks, _ = assembly.assemble(inst)
    for Mj in blocks[:4]:
        f = rrqr.qrcp_filter(Mj, tau)
        _check_factor(Mj, f, tol=1e-12)
        sv = np.linalg.svd(Mj, compute_uv=False)
        n = Mj.shape[1]
        lo = int(np.sum(sv > tau * sv[0] * 10 * np.sqrt(n)))
        hi = int(np.sum(sv > tau * sv[0] / (10 * np.sqrt(n))))
        assert lo <= f.rank <= hi
        # dropped columns: their residual after projection on the kept ones is below tau*|R00|
        if f.rank < min(Mj.shape):
            assert f.ratios[-1] <= tau


def test_qrcp_of_R0_chooses_same_pivots():
    """Column norms and all later trailing norms are invariant under an orthogonal
    left factor, so QRCP(M) and QRCP(R0) with R0 from an unpivoted QR pick the same columns."""
    inst = I.tiny("poisson2d")
    _, blocks, _ = assembly.assemble(inst)
    Mj = blocks[4]
    R0 = np.linalg.qr(Mj, mode="r")
    f1 = rrqr.qrcp_filter(Mj, 1e-8)
    f2 = rrqr.qrcp_filter(R0, 1e-8)
    assert f1.rank == f2.rank
    assert np.array_equal(f1.kept[: f1.rank - 2], f2.kept[: f1.rank - 2])
    assert np.allclose(f1.R[:10, :10], f2.R[:10, :10], rtol=1e-10, atol=1e-12 * f1.R[0, 0])
