"""Pins of the oracle's strong RRQR (Gu and Eisenstat's exchanges at the sigma-filter's rank).

Independent checks: rho from its QR-free definition (least-squares coefficients of the
trailing columns on the kept ones, their residual norms, and the diagonal of the inverse Gram
matrix), Kahan's matrix (where column pivoting keeps the identity order and reveals nothing),
the singular value bounds that a strong factorisation guarantees, and the growth of |det A|."""
import numpy as np
import pytest

from oracle import rrqr


def kahan(n, c, eps=1e-8):
    """Kahan's matrix diag(s^i) (I - c strict upper ones), s^2 + c^2 = 1, columns scaled by
    1 - eps k so that column pivoting keeps the identity order (every trailing norm ties)."""
    s = np.sqrt(1 - c * c)
    K = np.diag(s ** np.arange(n)) @ (np.triu(-c * np.ones((n, n)), 1) + np.eye(n))
    return K * (1 - eps * np.arange(n))[None, :]


def kahan_case(n=24):
    s = 0.3 ** (1 / (n - 1))
    return kahan(n, np.sqrt(1 - s * s)), s ** (n - 1.5)


def rho_by_definition(Mj, kept, rest):
    Mk, Mt = Mj[:, kept], Mj[:, rest]
    W, *_ = np.linalg.lstsq(Mk, Mt, rcond=None)
    gam2 = np.sum((Mt - Mk @ W) ** 2, axis=0)
    ginv = np.diag(np.linalg.inv(Mk.T @ Mk))
    return W * W + gam2[None, :] * ginv[:, None]


def test_rho_matches_its_qr_free_definition():
    rng = np.random.default_rng(1)
    Mj = rng.standard_normal((12, 7)) @ np.diag(np.logspace(0, -3, 7))
    perm = rng.permutation(7)
    r = 4
    got = rrqr.strong_measure(Mj, perm, r)
    want = rho_by_definition(Mj, perm[:r], perm[r:])
    assert np.allclose(got, want, rtol=1e-9, atol=1e-12)


def test_kahan_matrix_needs_an_exchange_and_gets_the_bounds():
    Kh, tau = kahan_case()
    n = Kh.shape[1]
    base = rrqr.qrcp_filter(Kh, tau)
    assert base.rank == n - 1 and np.array_equal(base.perm, np.arange(n))
    f = 2.0
    before = rrqr.strong_measure(Kh, base.perm, base.rank)
    assert before.max() > f * f                       # column pivoting is not strong here
    res, swaps, last = rrqr.strong_filter(Kh, tau, f)
    assert swaps >= 1 and res.rank == n - 1 and last <= f * f
    r = res.rank
    rest = np.array([k for k in range(n) if k not in set(res.kept)])
    assert rho_by_definition(Kh, res.kept, rest).max() <= f * f * (1 + 1e-9)
    # Gu-Eisenstat: sigma_i(A) >= sigma_i(M)/g and sigma_q(C) <= sigma_(r+q)(M) g
    g = np.sqrt(1 + f * f * r * (n - r))
    sv = np.linalg.svd(Kh, compute_uv=False)
    Rf = np.linalg.qr(Kh[:, np.concatenate([res.kept, rest])], mode="r")
    sa = np.linalg.svd(Rf[:r, :r], compute_uv=False)
    sc = np.linalg.svd(Rf[r:, r:], compute_uv=False)
    assert np.all(sa >= sv[:r] / g * (1 - 1e-12))
    assert np.all(sc <= sv[r:] * g * (1 + 1e-12))
    # column pivoting alone leaves |R_nn| = 0.3 against sigma_min = 1e-3: outside that bound
    assert abs(np.linalg.qr(Kh, mode="r")[-1, -1]) > sv[-1] * g
    # the kept factor is a QR of the kept columns with a positive diagonal
    assert np.allclose(res.Q @ res.R, Kh[:, res.kept], atol=1e-14)
    assert np.all(np.diag(res.R) > 0)


def test_every_exchange_grows_det_a_by_more_than_f():
    rng = np.random.default_rng(5)
    Mj = rng.standard_normal((30, 12)) @ np.diag(np.logspace(0, -8, 12)) @ rng.standard_normal((12, 12))
    base = rrqr.qrcp_filter(Mj, 1e-4)
    r, perm = base.rank, base.perm.copy()
    f = 1.05
    dets = []
    for _ in range(20):
        Rf = np.linalg.qr(Mj[:, perm], mode="r")
        dets.append(abs(np.prod(np.diag(Rf[:r, :r]))))
        rho = rrqr.strong_measure(Mj, perm, r)
        i, q, best = rrqr._argmax_first(rho)
        if best <= f * f:
            break
        perm[[i, r + q]] = perm[[r + q, i]]
    assert len(dets) >= 2, "this draw needs at least one exchange"
    assert all(b > a * f for a, b in zip(dets, dets[1:]))
    res, swaps, last = rrqr.strong_filter(Mj, 1e-4, f)
    assert swaps == len(dets) - 1 and last <= f * f


@pytest.mark.parametrize("name", ["poisson1d", "poisson2d"])
def test_strong_filter_keeps_column_pivoting_when_it_is_already_strong(name):
    from oracle import assembly
    from paper_2506_17626_amd import instances as I
    _, blocks, _ = assembly.assemble(I.tiny(name))
    for Mj in blocks:
        base = rrqr.qrcp_filter(Mj, 1e-8)
        res, swaps, last = rrqr.strong_filter(Mj, 1e-8, 2.0)
        if swaps == 0:
            assert np.array_equal(res.kept, base.kept) and np.array_equal(res.R, base.R) and last <= 4.0
        else:
            assert last <= 4.0 and res.rank == base.rank
