"""Pins of the oracle's precision form: narrow rounding and binary64 refinement."""
import numpy as np
import pytest
import torch

from oracle import assembly, forms, lsqr, rrqr
from paper_2506_17626_amd import instances as I


def test_bf16_rounding_matches_torch_and_hand_ties():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-20, 20, 5000),
                        [0.0, -0.0, 1.0, -1.0, 3.0e38, 1e-30]])
    ours = forms.round_bf16(x)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))
    # spacing of bfloat16 at 1 is 2^-7: ties go to the even mantissa
    assert forms.round_bf16(np.array([1 + 2.0**-8]))[0] == 1.0
    assert forms.round_bf16(np.array([1 + 3 * 2.0**-8]))[0] == 1 + 2.0**-6
    assert forms.round_bf16(np.array([1 + 2.0**-8 + 2.0**-20]))[0] == 1 + 2.0**-7
    assert np.array_equal(forms.round_f32(x), x.astype(np.float32))


def _system(name, tau):
    inst = I.tiny(name)
    rows, blocks, h = assembly.assemble(inst)
    facts = rrqr.filter_blocks(blocks, tau)
    A = lsqr.QForm(inst.N, rows, [f.Q for f in facts])
    return inst, rows, facts, A, h


def _dense_ls(A, h):
    D = np.stack([A.matvec(e) for e in np.eye(A.n)], axis=1)
    return np.linalg.lstsq(D, h, rcond=None)[0], np.linalg.cond(D)


@pytest.mark.parametrize("dtype,name,tau", [("f32", "heat3d", 1e-10), ("f32", "poisson1d", 1e-8),
                                            ("bf16", "poisson2d", 1e-1)])
def test_refinement_reaches_binary64_least_squares_solution(dtype, name, tau):
    inst, rows, facts, A, h = _system(name, tau)
    Al = forms.NarrowQForm(inst.N, rows, [f.Q for f in facts], dtype)
    ystar, kappa = _dense_ls(A, h)
    u_low = 2.0**-24 if dtype == "f32" else 2.0**-8
    assert kappa * u_low < 0.5, "refinement needs kappa * u_low < 1"
    y, info = forms.refine(A, Al, h, atol=1e-13, btol=1e-13, inner_tol=1e-6, max_outer=60)
    assert info.stop in (1, 2, 4)
    assert np.linalg.norm(y - ystar) <= 1e-9 * kappa * np.linalg.norm(ystar)
    assert info.outer >= 1


def test_refinement_alone_stalls_at_the_narrow_fixed_point():
    """Without the polish the gradient ||A^T r|| stalls near u_low ||A|| ||r||: the fixed point
    of refinement through the narrow operator solves A_low^T (h - A y) = 0."""
    inst, rows, facts, A, h = _system("heat3d", 1e-10)
    Al = forms.NarrowQForm(inst.N, rows, [f.Q for f in facts], "f32")
    y = np.zeros(A.n)
    for _ in range(8):
        d, _ = lsqr.lsqr(Al, h - A.matvec(y), atol=1e-10, btol=1e-10, maxit=20000)
        y = y + d
    r = h - A.matvec(y)
    eta = np.linalg.norm(A.rmatvec(r)) / (np.sqrt(A.n) * np.linalg.norm(r))
    y64, _ = lsqr.lsqr(A, h, atol=1e-14, btol=1e-14, maxit=20000)
    r64 = h - A.matvec(y64)
    eta64 = np.linalg.norm(A.rmatvec(r64)) / (np.sqrt(A.n) * np.linalg.norm(r64))
    assert 1e-10 < eta < 1e-6          # binary64 gradient stuck near the binary32 level
    assert eta64 < 1e-3 * eta          # far above what binary64 LSQR reaches


def test_refinement_first_step_error_follows_kappa_u_low():
    """One correction through the narrow operator lands within about kappa * u_low (relative) of
    the binary64 solution; further plain refinement steps do not get much closer (they stall at
    the narrow fixed point), which is why the precision form ends with a binary64 polish."""
    inst, rows, facts, A, h = _system("heat3d", 1e-10)
    Al = forms.NarrowQForm(inst.N, rows, [f.Q for f in facts], "bf16")
    ystar, kappa = _dense_ls(A, h)
    errs = []
    y = np.zeros(A.n)
    for _ in range(3):
        r = h - A.matvec(y)
        d, _ = lsqr.lsqr(Al, r, atol=1e-10, btol=1e-10, maxit=20000)
        y = y + d
        errs.append(np.linalg.norm(y - ystar) / np.linalg.norm(ystar))
    assert errs[0] <= 4 * kappa * 2.0**-8
    assert errs[0] > 1e-4                   # far from the binary64 solution
    assert errs[2] > 0.1 * errs[1]          # refinement alone stalls
    y2, info = forms.refine(A, Al, h, atol=1e-12, btol=1e-12, inner_tol=1e-6)
    assert info.polish_iters > 0
    assert np.linalg.norm(y2 - ystar) <= 1e-9 * kappa * np.linalg.norm(ystar)


def test_refinement_one_narrow_solve_to_the_rule_then_binary64_check():
    """The precision form's default: one narrow LSQR solve to the caller's own tolerance, then the
    binary64 test and, where it fails, the binary64 finish; the result is the binary64
    least-squares solution."""
    inst, rows, facts, A, h = _system("heat3d", 1e-10)
    Al = forms.NarrowQForm(inst.N, rows, [f.Q for f in facts], "f32")
    ystar, kappa = _dense_ls(A, h)
    y, info = forms.refine(A, Al, h, atol=1e-12, btol=1e-12, inner_tol=1e-12, max_outer=1)
    assert info.outer == 1 and info.stop in (1, 2, 4)
    assert np.linalg.norm(y - ystar) <= 1e-9 * kappa * np.linalg.norm(ystar)
    # from y = 0 the first narrow step is plain LSQR on h with the narrow operator
    yl, il = lsqr.lsqr(Al, h, atol=1e-12, btol=1e-12, maxit=100000, anorm=np.sqrt(A.n))
    assert info.inner_iters == il.iters


def test_refinement_warm_first_step_starts_from_the_given_coefficients():
    """A warm start enters the first narrow solve itself (LSQR on h from y0, its rule relative to
    ||h|| and ||y||): a start near the solution needs far fewer narrow iterations than y0 = 0."""
    inst, rows, facts, A, h = _system("heat3d", 1e-10)
    Al = forms.NarrowQForm(inst.N, rows, [f.Q for f in facts], "f32")
    ystar, kappa = _dense_ls(A, h)
    kw = dict(atol=1e-10, btol=1e-10, inner_tol=1e-10, max_outer=1)
    _, cold = forms.refine(A, Al, h, **kw)
    rng = np.random.default_rng(3)
    y0 = ystar * (1.0 + 1e-6 * rng.standard_normal(A.n))
    y, warm = forms.refine(A, Al, h, y0=y0, **kw)
    assert warm.stop in (1, 2, 4)
    assert np.linalg.norm(y - ystar) <= 1e-8 * kappa * np.linalg.norm(ystar)
    assert warm.inner_iters + warm.polish_iters < 0.5 * (cold.inner_iters + cold.polish_iters)
