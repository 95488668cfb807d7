"""Pins of the MLP reference, the single-precision emulation and the input generators."""
import numpy as np
import pytest

import workloads as w
from oracle import emulate, leads, mlp, rgf


# ---------------------------------------------------------------- MLP reference

def _small_net(seed=0):
    p = mlp.init_params(3, width=6, n_out=2, seed=seed)
    r = np.random.Generator(np.random.PCG64(seed + 1))
    for k in p:
        if k.startswith("b"):
            p[k] = r.normal(size=p[k].shape) * 0.1
    X = r.normal(size=(5, 3))
    T = r.normal(size=(5, 2))
    return p, X, T


@pytest.mark.parametrize("name", mlp.PARAM_NAMES)
def test_mlp_gradient_matches_finite_differences(name):
    p, X, T = _small_net()
    Y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, Y, T)
    num = mlp.numerical_grad(p, X, T, name)
    assert np.max(np.abs(g[name] - num)) < 1e-8 * max(1.0, np.max(np.abs(num)))


def test_adam_first_step_closed_form():
    """After one step the bias-corrected update is -lr g / (|g| + eps)."""
    p, X, T = _small_net(3)
    Y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, Y, T)
    p0 = {k: v.copy() for k, v in p.items()}
    m, v = mlp.adam_init(p)
    mlp.adam_step(p, g, m, v, 1, lr=1e-2)
    for k in p:
        assert np.allclose(p[k] - p0[k], -1e-2 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12, atol=1e-15)


def test_mlp_training_reduces_loss():
    r = np.random.Generator(np.random.PCG64(5))
    X = r.uniform(-1, 1, size=(64, 2))
    T = np.stack([np.sin(2 * X[:, 0]) * X[:, 1], np.cos(X[:, 0] + X[:, 1])], axis=1)
    p = mlp.init_params(2, width=16, seed=2)
    m, v = mlp.adam_init(p)
    l0 = mlp.mse(mlp.forward(p, X)[0], T)
    for t in range(1, 301):
        Y, c = mlp.forward(p, X)
        mlp.adam_step(p, mlp.backward(p, c, Y, T), m, v, t, lr=1e-2)
    assert mlp.mse(mlp.forward(p, X)[0], T) < 0.1 * l0


# ---------------------------------------------------------------- emulation

def _slab_problem(nb=5, b=64, E=0.2):
    dev = w.slab_device(nb, b, 2)
    L = leads.lead_self_energy(dev, 0, E, 1e-8)
    R = leads.lead_self_energy(dev, 1, E, 1e-8)
    Ad, Au, Al = rgf.assemble_blocks(dev, E, L.sigma_r, R.sigma_r)
    fl, fr = leads.fermi(E - 0.1, 0.025), leads.fermi(E + 0.1, 0.025)
    sig = [np.zeros_like(Ad[0]) for _ in Ad]
    sig[0] = sig[0] + leads.lesser_greater(L.gamma, fl)[0]
    sig[-1] = sig[-1] + leads.lesser_greater(R.gamma, fr)[0]
    return Ad, Au, Al, sig


def test_emulation_fp64_mode_is_rgf():
    Ad, Au, Al, sig = _slab_problem()
    R = emulate.retarded(Ad, Au, Al, "fp64")
    g, X, Gd, Gu, Gl = rgf.retarded(Ad, Au, Al)
    _, Ld, Lu = rgf.lesser(g, X, Gd, Gu, Al, sig)
    Le = emulate.lesser(R, Au, Al, sig, "fp64")
    assert np.allclose(np.array(R["Gd"]), np.array(Gd), rtol=0, atol=1e-13 * np.abs(np.array(Gd)).max())
    assert np.allclose(np.array(Le["Ld"]), np.array(Ld), rtol=0, atol=1e-13 * np.abs(np.array(Ld)).max())


def test_emulation_error_levels():
    Ad, Au, Al, sig = _slab_problem()
    ref = emulate.retarded(Ad, Au, Al, "fp64")
    refL = emulate.lesser(ref, Au, Al, sig, "fp64")

    def err(mode):
        R = emulate.retarded(Ad, Au, Al, mode)
        L = emulate.lesser(R, Au, Al, sig, mode)
        e = lambda a, b: np.linalg.norm(np.array(a) - np.array(b)) / np.linalg.norm(np.array(b))
        return max(e(R["Gd"], ref["Gd"]), e(R["Gu"], ref["Gu"])), max(e(L["Ld"], refL["Ld"]), e(L["Lu"], refL["Lu"]))

    r32, l32 = err("fp32")
    rr, lr = err("refine")
    assert 1e-8 < r32 < 1e-2 and 1e-8 < l32 < 1e-2     # single-precision products leave a visible error
    assert rr < 1e-8 and lr < 1e-7                      # one refinement per block restores it
    assert rr < 1e-2 * r32 and lr < 1e-2 * l32


# ---------------------------------------------------------------- generators

def test_generators_deterministic():
    a = w.slab_device(3, 40, 9)
    b = w.slab_device(3, 40, 9)
    assert np.array_equal(a.H_diag, b.H_diag) and np.array_equal(a.S_upper, b.S_upper)
    c = w.slab_device(3, 40, 10)
    assert not np.array_equal(a.H_diag, c.H_diag)


def test_slab_structure_b512():
    dev = w.slab_device(2, 512, 2)
    assert abs(np.mean(dev.H_diag[0] != 0) - 0.139) < 0.01
    assert abs(np.mean(dev.H_upper[0] != 0) - 0.085) < 0.01
    assert np.allclose(dev.H_diag[0], dev.H_diag[0].conj().T)
    # S = I + P with 0 <= P, ||P|| <= 0.05 on the full matrix
    N = 2 * 512
    S = np.zeros((N, N), complex)
    S[:512, :512] = dev.S_diag[0]
    S[512:, 512:] = dev.S_diag[1]
    S[:512, 512:] = dev.S_upper[0]
    S[512:, :512] = dev.S_upper[0].conj().T
    ev = np.linalg.eigvalsh(S)
    assert ev.min() >= 1.0 - 1e-12 and ev.max() <= 1.05 + 1e-12


def test_scattering_self_energies_properties():
    dev = w.scattering_self_energies(w.random_device(3, 6, 1), 3)
    for i in range(3):
        sl, sg, sr = dev.sig_l[i], dev.sig_g[i], dev.sig_r[i]
        assert np.linalg.norm(sl + sl.conj().T) < 1e-15
        assert abs(np.linalg.norm(sl, 2) - 0.01) < 1e-12
        assert np.linalg.eigvalsh(-1j * sl).min() > -1e-15
        assert np.linalg.eigvalsh(1j * sg).min() > -1e-15
        assert np.allclose(sr - sr.conj().T, sg - sl)


def test_k_device_hermitian_and_periodic_in_k():
    dev = w.slab_device(2, 64, 2)
    d0 = w.k_device(dev, 7, 0.3)
    d1 = w.k_device(dev, 7, 0.3 + 2 * np.pi)
    assert np.allclose(d0.H_diag, d1.H_diag)
    assert np.allclose(d0.H_diag[1], d0.H_diag[1].conj().T)
    assert np.array_equal(d0.H_upper, dev.H_upper)
