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


def test_standardisation_and_loss_kernels_match_numpy(learned):
    import torch
    r = np.random.Generator(np.random.PCG64(11))
    X = (r.normal(size=(20000, 6)) * np.array([1, 3, 0.1, 10, 2, 5]) + np.array([0, 1, -2, 4, 0.5, 7])).astype(
        np.float32)
    net = learned.MLP(seed=0)
    Xt = torch.from_numpy(X).cuda()
    net.set_normalisation(Xt)
    mu, sd = net.mu.cpu().numpy(), net.sd.cpu().numpy()
    assert np.allclose(mu, X.astype(np.float64).mean(0), rtol=1e-6, atol=1e-6)
    assert np.allclose(sd, X.astype(np.float64).std(0, ddof=1), rtol=1e-6)
    Xn = net._norm(Xt).cpu().numpy()
    assert np.allclose(Xn, (X - mu) / sd, rtol=1e-6, atol=1e-6)
    Y = r.normal(size=(5000, 2)).astype(np.float32)
    T = r.normal(size=(5000, 2)).astype(np.float32)
    got = net.loss(torch.from_numpy(Y).cuda(), torch.from_numpy(T).cuda()).item()
    assert abs(got - np.mean((Y.astype(np.float64) - T) ** 2)) < 1e-12 * 10


def test_signed_log_and_its_inverse(learned):
    import torch
    x = np.concatenate([np.linspace(-1e4, 1e4, 1001), [0.0, -0.0, 1e-30, -1e-30]]).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    y = learned.signed_log(xt).cpu().numpy()
    ref = np.sign(x) * np.log1p(np.abs(x.astype(np.float64)))
    assert np.allclose(y, ref, rtol=5e-7, atol=1e-30)
    back = learned.signed_log(learned.signed_log(xt), inverse=True).cpu().numpy()
    assert np.allclose(back, x, rtol=1e-5, atol=1e-30)


def test_mode_transforms_match_numpy(learned):
    import torch
    from paper_2602_03438_amd import binding as nb
    r = np.random.Generator(np.random.PCG64(12))
    n, b = 3, 40
    T = r.normal(size=(n, b, b)) + 1j * r.normal(size=(n, b, b))
    out = torch.empty(n * b, 2, dtype=torch.float32, device="cuda")
    Tt = torch.from_numpy(T).cuda()
    nb.check(nb.lib().negf_mode_diag(n, b, nb._ptr(Tt), nb._ptr(out), nb._stream()))
    d = np.diagonal(T, axis1=1, axis2=2).reshape(-1)
    assert np.allclose(out.cpu().numpy(), np.stack([d.real, d.imag], 1).astype(np.float32))
    U = r.normal(size=(b, b)) + 1j * r.normal(size=(b, b))
    y = r.normal(size=(n * b, 2)).astype(np.float32)
    basis = learned.GPUBasis.__new__(learned.GPUBasis)
    basis.b = b
    basis.U = torch.from_numpy(U).cuda()
    seeds = basis.seeds(torch.from_numpy(y).cuda()).cpu().numpy()
    x = (y[:, 0].astype(np.float64) + 1j * y[:, 1]).reshape(n, b)
    ref = np.stack([U @ np.diag(x[p]) @ U.conj().T for p in range(n)])
    assert np.linalg.norm(seeds - ref) < 1e-13 * np.linalg.norm(ref)


def test_training_checkpoint_round_trip(learned, tmp_path):
    """Parameters, Adam moments, step and standardisation survive save / load: a
    restored network takes exactly the same next step as the original."""
    import torch
    a, X, T = _setup(learned, n=512, H=64, seed=21)
    a.set_normalisation(X)
    for _ in range(3):
        Y, c = a.forward(X)
        a.backward(c, Y, T)
        a.adam(lr=1e-3)
    path = str(tmp_path / "mlp.safetensors")
    a.save(path)
    b = learned.MLP(seed=99, width=64)
    b.load(path)
    assert b.t == a.t == 3
    for net in (a, b):
        Y, c = net.forward(X)
        net.backward(c, Y, T)
        net.adam(lr=1e-3)
    for k in a.p:
        assert torch.equal(a.p[k], b.p[k]) and torch.equal(a.m[k], b.m[k]) and torch.equal(a.v[k], b.v[k]), k
    wrong = learned.MLP(seed=0, width=32)
    with pytest.raises(ValueError):
        wrong.load(path)
