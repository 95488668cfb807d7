"""GPU parity of the kernel-level entry points (complex products, inversion)."""
import numpy as np
import pytest

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


def _op(x, o):
    return x if o == "N" else np.conj(np.swapaxes(x, -1, -2))


@pytest.mark.parametrize("prec", [0, 2])
@pytest.mark.parametrize("opa", ["N", "C"])
@pytest.mark.parametrize("opb", ["N", "C"])
@pytest.mark.parametrize("M,N,K", [(64, 64, 64), (37, 71, 19), (130, 100, 133), (8, 8, 8), (1, 5, 3)])
def test_zgemm_fp64_parity(nb, opa, opb, M, N, K, prec):
    """prec 0: four real products per complex product; 2: three (Gauss)."""
    import torch
    r = np.random.Generator(np.random.PCG64(M * 1000 + N * 10 + K))
    batch = 3
    A = _rand(r, (batch, M, K) if opa == "N" else (batch, K, M))
    B = _rand(r, (batch, K, N) if opb == "N" else (batch, N, K))
    C0 = _rand(r, (batch, M, N))
    alpha, beta = 0.7 - 0.3j, -1.1 + 0.4j
    ref = alpha * (_op(A, opa) @ _op(B, opb)) + beta * C0
    Ct = torch.from_numpy(C0.copy()).cuda()
    nb.zgemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), Ct, opa, opb, alpha, beta, prec=prec)
    got = Ct.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-14 * max(1, np.sqrt(K)), err


@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("opa,opb", [("N", "N"), ("C", "N"), ("N", "C"), ("C", "C")])
@pytest.mark.parametrize("M,N,K", [(200, 130, 77), (128, 256, 64), (128, 128, 48), (128, 64, 16)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_zgemm_tile_shapes(nb, tile, opa, opb, M, N, K, prec):
    """Ragged sizes and sizes that are whole tiles (the unchecked full-tile
    path), with an odd and a single K-step among the latter."""
    import torch
    r = np.random.Generator(np.random.PCG64(M + N + K + tile))
    A = _rand(r, (2, M, K) if opa == "N" else (2, K, M))
    B = _rand(r, (2, K, N) if opb == "N" else (2, N, K))
    C0 = _rand(r, (2, M, N))
    ref = (0.5 + 0.25j) * (_op(A, opa) @ _op(B, opb)) - C0
    Ct = torch.from_numpy(C0.copy()).cuda()
    nb.zgemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), Ct, opa, opb, 0.5 + 0.25j, -1.0, prec=prec,
             tile=tile)
    err = np.linalg.norm(Ct.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err < (1e-5 if prec == 1 else 1e-13), err


@pytest.mark.parametrize("prec", [0, 2])
def test_zgemm_fp64_b1024_largest_block(nb, prec):
    """The largest block the library accepts: 64 K-steps in one tile."""
    import torch
    r = np.random.Generator(np.random.PCG64(6))
    A = _rand(r, (2, 1024, 1024))
    B = _rand(r, (2, 1024, 1024))
    got = nb.zgemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), prec=prec).cpu().numpy()
    ref = A @ B
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-14


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("tile", [1, 2, 4, 5, 6])
@pytest.mark.parametrize("K", [1040, 2048])
@pytest.mark.parametrize("opa,opb", [("N", "N"), ("C", "N"), ("C", "C")])
def test_zgemm_long_k_full_tiles(nb, K, tile, prec, opa, opb):
    """Whole-tile sizes with more than 64 K-steps: every K-step has to be
    taken (the full-tile path walks the steps in order for dense operands)."""
    import torch
    r = np.random.Generator(np.random.PCG64(K + 10 * tile + prec))
    M, N = 128, 64
    A = _rand(r, (2, M, K) if opa == "N" else (2, K, M))
    B = _rand(r, (2, K, N) if opb == "N" else (2, N, K))
    C0 = _rand(r, (2, M, N))
    ref = (_op(A, opa) @ _op(B, opb)) + (0.5 - 0.5j) * C0
    Ct = torch.from_numpy(C0.copy()).cuda()
    nb.zgemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), Ct, opa, opb, 1.0, 0.5 - 0.5j, prec=prec,
             tile=tile)
    err = np.linalg.norm(Ct.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err < (1e-5 if prec == 1 else 1e-13), err


@pytest.mark.parametrize("prec", [0, 2])
def test_zgemm_fp64_b512_batched(nb, prec):
    import torch
    r = np.random.Generator(np.random.PCG64(5))
    A = _rand(r, (4, 512, 512))
    B = _rand(r, (4, 512, 512))
    got = nb.zgemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), prec=prec).cpu().numpy()
    ref = A @ B
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-14


@pytest.mark.parametrize("n", [8, 72, 130, 512])
@pytest.mark.parametrize("prec", [0, 2, 1])
@pytest.mark.parametrize("tile", [1, 2, 4, 6])
def test_zgemm_skew_product(nb, n, prec, tile):
    """A X A^H + S with X and S anti-Hermitian, computed as an anti-Hermitian
    product (prec + 4): upper triangle computed, lower mirrored."""
    import torch
    r = np.random.Generator(np.random.PCG64(n + 7 * prec + tile))
    A = _rand(r, (3, n, n))
    X = _rand(r, (3, n, n))
    X = X - np.conj(np.swapaxes(X, -1, -2))
    S = _rand(r, (3, n, n))
    S = S - np.conj(np.swapaxes(S, -1, -2))
    AX = A @ X
    ref = AX @ np.conj(np.swapaxes(A, -1, -2)) + S
    Ct = torch.from_numpy(S.copy()).cuda()
    nb.zgemm(torch.from_numpy(AX).cuda(), torch.from_numpy(A).cuda(), Ct, "N", "C", 1.0, 1.0, prec=prec + 4,
             tile=tile)
    got = Ct.cpu().numpy()
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < (1e-5 if prec == 1 else 1e-13), err
    assert np.array_equal(got, -np.conj(np.swapaxes(got, -1, -2))) or n == 0 or \
        np.array_equal(np.tril(got, -1), np.tril(-np.conj(np.swapaxes(got, -1, -2)), -1))


def test_zgemm_fp32_products(nb):
    import torch
    r = np.random.Generator(np.random.PCG64(6))
    A = _rand(r, (2, 200, 150))
    B = _rand(r, (2, 150, 90))
    got = nb.zgemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), prec=1).cpu().numpy()
    ref = A @ B
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    # single-precision operands and accumulation: ~1e-7 relative, not double accuracy
    assert 1e-9 < err < 1e-5, err


@pytest.mark.parametrize("n", [1, 5, 8, 16, 33, 100, 130, 300, 512, 700, 1000, 1024])
@pytest.mark.parametrize("panel", [16, 32])
def test_zinv_parity(nb, n, panel):
    import torch
    r = np.random.Generator(np.random.PCG64(n + panel))
    M = _rand(r, (3, n, n)) + 2.0 * np.sqrt(n) * np.eye(n) * np.array([1, 1j, -1])[:, None, None]
    # a row permutation makes pivoting necessary
    M = np.ascontiguousarray(M[:, r.permutation(n), :])
    out, info = nb.zinv(torch.from_numpy(M).cuda(), panel)
    got = out.cpu().numpy()
    ref = np.linalg.inv(M)
    assert np.all(info.cpu().numpy() == 0)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    assert err < 1e-13, err
    eye_err = np.linalg.norm(M @ got - np.eye(n)) / np.sqrt(n)
    assert eye_err < 1e-12


def test_zinv_pivoting_needed(nb):
    """A matrix with a zero leading entry is only invertible with row exchanges."""
    import torch
    M = np.array([[0, 1, 2], [3, 0, 1], [1, 1, 0]], dtype=np.complex128)[None]
    out, info = nb.zinv(torch.from_numpy(M).cuda(), 16)
    assert np.allclose(out.cpu().numpy()[0], np.linalg.inv(M[0]), atol=1e-14)


@pytest.mark.parametrize("n", [64, 200, 512, 1024])
def test_zinv_scaled_permutation(nb, n):
    """One non-zero per row and column, anywhere in the matrix: every pivot has
    to be the single non-zero of its column among all remaining rows (any other
    choice is a zero pivot), so this checks the pivot search across every
    wavefront of the workgroup, and the interchanges across super-panels."""
    import torch
    r = np.random.Generator(np.random.PCG64(n))
    perm = r.permutation(n)
    vals = np.exp(r.uniform(-5, 5, (2, n))) * np.exp(2j * np.pi * r.uniform(size=(2, n)))
    M = np.zeros((2, n, n), dtype=np.complex128)
    M[0, np.arange(n), perm] = vals[0]
    M[1, perm, np.arange(n)] = vals[1]
    out, info = nb.zinv(torch.from_numpy(M).cuda(), 16)
    assert np.all(info.cpu().numpy() == 0)
    got = out.cpu().numpy()
    for k in range(2):
        ref = np.linalg.inv(M[k])
        assert np.linalg.norm(got[k] - ref) / np.linalg.norm(ref) < 1e-14


def test_zinv_reports_singular_and_nonfinite(nb):
    import torch
    r = np.random.Generator(np.random.PCG64(9))
    M = _rand(r, (3, 20, 20))
    M[1, :, 3] = 0.0                    # exactly singular
    M[2, 4, 4] = np.nan                 # non-finite
    out, info = nb.zinv(torch.from_numpy(M).cuda(), 16)
    info = info.cpu().numpy()
    assert info[0] == nb.NEGF_OK
    assert info[1] == nb.NEGF_ESINGULAR
    assert info[2] in (nb.NEGF_ENONFINITE, nb.NEGF_ESINGULAR)
    assert np.allclose(out.cpu().numpy()[0], np.linalg.inv(M[0]), atol=1e-12)
