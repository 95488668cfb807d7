"""GPU energy convolution (negf_energy_convolution) and layout change
(negf_transpose) against the oracle (oracle/econv.py, the plain sum)."""
import numpy as np
import pytest

from oracle import econv as oec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2602_03438_amd import binding
    binding.lib()
    return binding


def _rand(r, shape):
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


# (n_e, n_w, k0, n_el): every transform length from 16 to 4096 (and so every
# elements-per-workgroup choice), ragged element counts (47 at L = 2048: 24 tiles of
# two, so the XCD-contiguous order with a ragged last tile), one- and two-sided kernels
CASES = [(5, 3, 1, 7), (9, 20, 0, 33), (40, 25, 12, 100), (100, 29, 28, 37), (200, 57, 3, 64), (300, 211, 105, 41),
         (512, 513, 256, 19), (1024, 1024, 512, 24), (700, 900, 450, 47), (1500, 1200, 600, 5), (2048, 2049, 1024, 3)]


@pytest.mark.parametrize("n_e,n_w,k0,n_el", CASES)
def test_energy_convolution_matches_oracle(nb, n_e, n_w, k0, n_el):
    import torch
    r = np.random.Generator(np.random.PCG64(n_e * 7 + n_w))
    G = _rand(r, (n_e, n_el))
    W = _rand(r, (n_w, n_el))
    scale = 0.3 - 0.7j
    got = nb.energy_convolution(torch.from_numpy(G).cuda(), torch.from_numpy(W).cuda(), k0, scale).cpu().numpy()
    ref = oec.energy_convolution(G, W, k0, scale)
    # an FFT convolution of length L is accurate to ~eps log2(L) relative to sum_k |G||W|
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-13, err


def test_energy_convolution_many_elements_xcd_order(nb):
    """Enough element tiles (a multiple of 8) for the XCD-contiguous tile order."""
    import torch
    r = np.random.Generator(np.random.PCG64(3))
    n_e, n_w, k0, n_el = 120, 80, 40, 8 * 8 * 37
    G, W = _rand(r, (n_e, n_el)), _rand(r, (n_w, n_el))
    got = nb.energy_convolution(torch.from_numpy(G).cuda(), torch.from_numpy(W).cuda(), k0).cpu().numpy()
    ref = oec.energy_convolution(G, W, k0)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-13


def test_energy_convolution_identity_kernel_is_exact_copy(nb):
    """W = delta at k0 returns scale * G (the transforms of a delta are exact up to rounding)."""
    import torch
    r = np.random.Generator(np.random.PCG64(4))
    G = _rand(r, (333, 50))
    W = np.zeros((64, 50), complex)
    W[17] = 1.0
    got = nb.energy_convolution(torch.from_numpy(G).cuda(), torch.from_numpy(W).cuda(), 17, 2.0).cpu().numpy()
    assert np.max(np.abs(got - 2.0 * G)) < 1e-13 * np.max(np.abs(G))


def test_energy_convolution_rejects(nb):
    import torch
    G = torch.zeros(3000, 2, dtype=torch.complex128, device="cuda")
    W = torch.zeros(1200, 2, dtype=torch.complex128, device="cuda")
    with pytest.raises(nb.NegfError):
        nb.energy_convolution(G, W, 0)                    # 3000 + 1200 - 1 > 4096
    with pytest.raises(nb.NegfError):
        nb.energy_convolution(G[:10].contiguous(), W[:5].contiguous(), 5)   # k0 >= n_w


@pytest.mark.parametrize("rows,cols", [(1, 1), (7, 33), (64, 64), (1000, 37), (33, 2049)])
def test_transpose_matches_numpy(nb, rows, cols):
    import torch
    r = np.random.Generator(np.random.PCG64(rows + cols))
    X = _rand(r, (rows, cols))
    got = nb.transpose(torch.from_numpy(X).cuda()).cpu().numpy()
    assert np.array_equal(got, oec.to_element_major(X))


def test_output_tensors_are_checked(nb):
    """The helpers refuse outputs that the kernels would write past (the library
    itself only sees pointers)."""
    import torch
    G = torch.zeros(8, 3, dtype=torch.complex128, device="cuda")
    W = torch.zeros(4, 3, dtype=torch.complex128, device="cuda")
    with pytest.raises(nb.NegfError):
        nb.energy_convolution(G, W, 1, out=torch.zeros(8, 2, dtype=torch.complex128, device="cuda"))
    with pytest.raises(nb.NegfError):
        nb.energy_convolution(G, W, 1, out=torch.zeros(8, 3, dtype=torch.complex64, device="cuda"))
    with pytest.raises(nb.NegfError):
        nb.transpose(G, out=torch.zeros(8, 3, dtype=torch.complex128, device="cuda"))
