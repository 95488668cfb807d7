"""GPU MLP kernels (learned lead initialiser) against the float64 oracle."""
import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def learned():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2602_03438_amd import binding, learned as L
    binding.lib()
    return L


def _to_np(p):
    return {k: v.double().cpu().numpy() for k, v in p.items()}


def _setup(L, n=300, F=6, H=64, O=2, seed=1):
    import torch
    net = L.MLP(seed=seed, n_in=F, width=H, n_out=O)
    r = np.random.Generator(np.random.PCG64(seed + 7))
    for k in ("b1", "b2", "b3"):
        net.p[k] = torch.from_numpy(r.normal(size=net.p[k].shape).astype(np.float32) * 0.1).cuda()
    X = torch.from_numpy(r.normal(size=(n, F)).astype(np.float32)).cuda()
    T = torch.from_numpy(r.normal(size=(n, O)).astype(np.float32)).cuda()
    return net, X, T


def test_mlp_forward_backward_match_oracle(learned):
    net, X, T = _setup(learned)
    Y, cache = net.forward(X)
    g = net.backward(cache, Y, T)
    p64 = _to_np(net.p)
    X64 = X.double().cpu().numpy()          # mu = 0, sd = 1: normalisation is the identity here
    Y64, c64 = omlp.forward(p64, X64)
    g64 = omlp.backward(p64, c64, Y64, T.double().cpu().numpy())
    assert np.max(np.abs(Y.double().cpu().numpy() - Y64)) < 1e-5 * max(1.0, np.abs(Y64).max())
    for k in omlp.PARAM_NAMES:
        got = g[k].double().cpu().numpy()
        ref = g64[k]
        assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref) + 1e-9, k


def test_mlp_adam_matches_oracle(learned):
    net, X, T = _setup(learned, seed=3)
    Y, cache = net.forward(X)
    net.backward(cache, Y, T)
    p0 = _to_np(net.p)
    g = _to_np(net.g)
    net.adam(lr=1e-2)
    m, v = omlp.adam_init(p0)
    p1 = {k: x.copy() for k, x in p0.items()}
    omlp.adam_step(p1, g, m, v, 1, lr=1e-2)
    for k in p1:
        assert np.max(np.abs(net.p[k].double().cpu().numpy() - p1[k])) < 1e-6


def test_mlp_bf16_inference_close_to_fp32(learned):
    net, X, T = _setup(learned, n=1000, H=256, seed=5)
    Y32, _ = net.forward(X)
    Yb = net.infer_bf16(X)
    err = (Yb - Y32).norm() / Y32.norm()
    assert float(err) < 3e-2


def test_mlp_training_reduces_loss(learned):
    import torch
    net, X, _ = _setup(learned, n=4096, H=64, seed=9)
    T = torch.stack([torch.sin(X[:, 0]) * X[:, 1], torch.cos(X[:, 2])], dim=1).contiguous()
    losses = net.train(X, T, epochs=30, batch=512, lr=3e-3)
    assert losses[-1] < 0.2 * losses[0]
