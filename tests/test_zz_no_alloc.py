"""negf_rgf_lesser_greater_static (the allocation-free variant: the library's
own static scratch instead of a workspace) against negf_rgf_lesser_greater on
the same inputs, through the C ABI: two calls in a row, the second with a
smaller input, then a call that needs several chunks of the scratch, and the
synchronous NEGF_ENOMEM of a point that does not fit."""
import numpy as np
import pytest

import workloads as w

pytestmark = pytest.mark.gpu

KEYS = ("GR_diag", "GR_upper", "GR_lower", "GL_diag", "GL_upper", "GG_diag", "GG_upper")


@pytest.fixture(scope="module")
def nb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2602_03438_amd import binding
    binding.lib()
    return binding


def _problem(nb, dev, energies):
    return nb.Problem(nb.DeviceOnGPU(dev), energies, eta=1e-8, mu_l=0.1, mu_r=-0.1, kT=0.025)


def _same(nb, probs, opts=None, greater=True):
    """Both entry points on the same problems; every output bit-identical (the
    same kernels, the same per-point arithmetic, only the scratch differs)."""
    import torch
    ref = nb.rgf_lesser_greater(probs, greater=greater, opts=opts)
    got = nb.rgf_lesser_greater_static(probs, greater=greater, opts=opts)
    torch.cuda.synchronize()
    assert got["status"] == nb.NEGF_OK, nb.status_string(got["status"])
    assert torch.equal(got["info"], ref["info"])
    for key in KEYS:
        if ref["flat"].get(key) is None:
            continue
        for q in range(len(probs)):
            assert torch.equal(got[key][q], ref[key][q]), (key, q)
    return got


def test_static_scratch_two_calls_second_smaller(nb):
    dev = w.slab_device(4, 64, 2)
    w.scattering_self_energies(dev, 3)
    first = _same(nb, [_problem(nb, dev, np.array([-0.95, -0.15, 0.25, 0.6, 1.0]))])
    assert np.all(first["info"].cpu().numpy() == 0)
    # the second call is smaller and of another shape: nothing of the first call's scratch leaks in
    small = w.slab_device(3, 40, 5)
    second = _same(nb, [_problem(nb, small, np.array([-0.4, 0.7]))], greater=False)
    assert np.all(second["info"].cpu().numpy() == 0)


def test_static_scratch_in_chunks(nb):
    """Nb = 60 blocks of b = 128: ~24 MiB of workspace per point, so 24 points go
    through the scratch in chunks (the workspace call takes them in one)."""
    dev = w.slab_device(60, 128, 2)
    energies = np.linspace(-1.2, 1.2, 24)
    _same(nb, [_problem(nb, dev, energies)], greater=False)


def test_static_scratch_rejects_what_does_not_fit(nb):
    import torch
    b, nbk = 512, 60
    H_d = torch.zeros(nbk, b, b, dtype=torch.complex128, device="cuda")
    H_u = torch.zeros(nbk - 1, b, b, dtype=torch.complex128, device="cuda")
    g = nb.DeviceOnGPU.__new__(nb.DeviceOnGPU)
    g.nb, g.b = nbk, b
    g.H_diag, g.H_upper = H_d, H_u
    g.S_diag = g.S_upper = g.sig_r = g.sig_l = g.sig_g = None
    prob = nb.Problem(g, np.array([0.1]), eta=1e-8)
    # outputs of one point (1.2 GB) are allocated by the caller; the call itself must refuse
    res = nb.rgf_lesser_greater_static([prob])
    assert res["status"] == nb.NEGF_ENOMEM
    # a requested batch that does not fit is refused the same way
    dev = w.slab_device(60, 128, 2)
    p2 = _problem(nb, dev, np.linspace(-1, 1, 12))
    res = nb.rgf_lesser_greater_static([p2], opts=nb.make_options(batch=12))
    assert res["status"] == nb.NEGF_ENOMEM
    torch.cuda.synchronize()
