"""GPU perceptron kernels (binary32) against the binary64 oracle: forward activations,
gradients of every parameter (relative to the gradient's scale), the Adam update."""
import numpy as np
import pytest
import torch

from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rfm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_17626_amd import rfm as lib
    return lib


def _dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("n_in,H,n_out,batch", [(12, 64, 300, 37), (12, 512, 5000, 256), (7, 96, 65, 5)])
def test_forward_backward_match_oracle(rfm, n_in, H, n_out, batch):
    rng = np.random.default_rng(n_out)
    P = mlp.init_params(n_in, H, n_out, seed=1)
    for k in ("b1", "b2", "b3"):
        P[k] = rng.standard_normal(P[k].shape) * 0.1
    # use the binary32-rounded parameters and data on both sides
    P = {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}
    X = rng.uniform(-1, 1, (batch, n_in)).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((batch, n_out)).astype(np.float32).astype(np.float64)
    H1o, H2o, Yo = mlp.forward(P, X)
    Lo, Go = mlp.backward(P, X, T)
    Pd = {k: _dev32(v) for k, v in P.items()}
    Gd = {k: torch.zeros_like(v) for k, v in Pd.items()}
    Xd, Td = _dev32(X), _dev32(T)
    H1, H2, Y = rfm.rfm_mlp_forward(Pd, Xd)
    loss = rfm.rfm_mlp_backward(Pd, Gd, Xd, H1, H2, Y, Td)
    torch.cuda.synchronize()
    for got, ref in ((H1, H1o), (H2, H2o), (Y, Yo)):
        assert np.max(np.abs(got.cpu().numpy() - ref)) <= 1e-5 * max(1.0, np.abs(ref).max())
    assert abs(float(loss.item()) - Lo) <= 1e-5 * Lo
    for k in Go:
        g = Gd[k].cpu().numpy()
        scale = np.abs(Go[k]).max()
        assert np.max(np.abs(g - Go[k])) <= 1e-4 * scale, k


def test_adam_step_matches_oracle(rfm):
    rng = np.random.default_rng(2)
    p = rng.standard_normal(1000).astype(np.float32)
    g = rng.standard_normal(1000).astype(np.float32)
    m = (rng.standard_normal(1000) * 0.1).astype(np.float32)
    v = (rng.uniform(0, 1, 1000)).astype(np.float32)
    pd, gd, md, vd = (_dev32(a) for a in (p, g, m, v))
    rfm.rfm_adam_step(pd, gd, md, vd, step=7, lr=1e-2)
    po, mo, vo = mlp.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                               v.astype(np.float64), 7, lr=1e-2)
    torch.cuda.synchronize()
    assert np.allclose(pd.cpu().numpy(), po, rtol=1e-5, atol=1e-6)
    assert np.allclose(md.cpu().numpy(), mo, rtol=1e-6, atol=1e-7)
    assert np.allclose(vd.cpu().numpy(), vo, rtol=1e-6, atol=1e-7)


def test_gather_rows(rfm):
    src = torch.arange(40, dtype=torch.float32, device="cuda").reshape(10, 4)
    idx = torch.tensor([3, 0, 9, 3], dtype=torch.int32, device="cuda")
    out = rfm.rfm_gather_rows(idx, src, torch.empty(4, 4, device="cuda"))
    assert torch.equal(out, src[idx.long()])
