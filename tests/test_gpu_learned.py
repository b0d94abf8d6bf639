"""Learned warm start on the GPU: trained by the library's own kernels on solves the method
generates; on held-out members of the family the warm-started LSQR reaches the cold start's
solution, starts from a smaller residual, and its iteration count is measured against the cold
start (the gain is small: LSQR's iteration count here is set by the weak directions, which a
start that is tens of percent off does not shorten); a start whose residual exceeds that of the
zero start is rejected and the solve is then the cold one, bit for bit."""
import numpy as np
import pytest
import torch

from paper_2506_17626_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_17626_amd import learned, rfm
    return rfm, learned


def test_warm_start_gains_over_cold_start(lib):
    rfm, learned = lib
    inst = I.poisson2d(S=3, K=40, n=7, nb=21, seed=0, name="poisson2d_family_tiny")
    plan = rfm.plan_instance(inst)
    prob = rfm.problem_tensors(inst)
    M, h = rfm.rfm_assemble(plan, prob)
    fact = rfm.rfm_rrqr_filter(plan, M, 1e-8)
    maxfreq = 2
    train = I.poisson2d_family_params(512, seed=11, maxfreq=maxfreq)
    test = I.poisson2d_family_params(12, seed=12, maxfreq=maxfreq)
    ts = learned.solve_members(plan, fact, inst, prob, train, maxfreq, tol=1e-10, maxit=20000)
    assert np.all(np.isin(ts.stops, (1, 2, 4)))
    model = learned.train_warm_start(ts, hidden=64, epochs=300, batch=64, lr=3e-3, seed=1, maxfreq=maxfreq)
    print(f"  loss first {model.loss_history[0]:.3e} last {model.loss_history[-1]:.3e}", flush=True)
    assert model.loss_history[-1] < 0.2 * model.loss_history[0]
    Ht = learned.family_rhs(inst, prob, test)
    Y0 = model.starts(plan, fact, test)
    cold, warm, start_rel, rejected = [], [], [], 0
    for b in range(len(test)):
        hb = Ht[:, b].contiguous()
        yc, ic = rfm.rfm_lsqr_solve(plan, fact, hb, atol=1e-8, btol=1e-8, maxit=20000)
        y0 = Y0[:, b].contiguous()
        yw, iw = rfm.rfm_lsqr_solve(plan, fact, hb, y0=y0, atol=1e-8, btol=1e-8, maxit=20000)
        assert ic.stop in (1, 2, 4) and iw.stop in (1, 2, 4)
        start_rel.append(float(torch.linalg.norm(y0 - yc) / torch.linalg.norm(yc)))
        if iw.warm_rejected:
            # a start whose residual exceeds ||h|| falls back to the cold start exactly
            rejected += 1
            assert iw.iters == ic.iters and torch.equal(yw, yc)
            continue
        assert torch.linalg.norm(yw - yc) <= 1e-4 * torch.linalg.norm(yc)
        cold.append(ic.iters)
        warm.append(iw.iters)
    print(f"  start error vs solution {np.round(start_rel, 3).tolist()}\n  rejected starts {rejected}\n"
          f"  accepted: cold iterations {cold}\n  accepted: warm iterations {warm}", flush=True)
    assert np.median(start_rel) < 1.0         # the network predicts part of the solution
    if warm:
        assert np.mean(warm) <= 1.05 * np.mean(cold)


def test_harmful_warm_start_is_rejected(lib):
    rfm, learned = lib
    inst = I.tiny("poisson2d")
    plan = rfm.plan_instance(inst)
    prob = rfm.problem_tensors(inst)
    M, h = rfm.rfm_assemble(plan, prob)
    fact = rfm.rfm_rrqr_filter(plan, M, 1e-8)
    yc, ic = rfm.rfm_lsqr_solve(plan, fact, h, atol=1e-10, btol=1e-10, maxit=20000)
    bad = torch.full_like(yc, 1e6)
    yw, iw = rfm.rfm_lsqr_solve(plan, fact, h, y0=bad, atol=1e-10, btol=1e-10, maxit=20000)
    assert iw.warm_rejected == 1 and iw.iters == ic.iters
    assert torch.equal(yw, yc)
