"""Pins of the lead self-energy oracle (decimation) against closed forms and brute force."""
import cmath

import numpy as np
import pytest

import workloads as w
from oracle import dense, leads


def chain_surface_closed_form(z, eps=0.0, t=1.0):
    """Root of t^2 g^2 - (z - eps) g + 1 = 0 with |t g| < 1 (retarded, decaying)."""
    w_ = z - eps
    s = cmath.sqrt(w_ * w_ - 4 * t * t)
    r1 = (w_ + s) / (2 * t * t)
    r2 = (w_ - s) / (2 * t * t)
    return r1 if abs(t * r1) < 1 else r2


@pytest.mark.parametrize("E", [-2.5, -1.7, -0.9, -0.3, 0.4, 1.1, 1.95, 2.6])
@pytest.mark.parametrize("side", [0, 1])
def test_chain_surface_gf_closed_form(E, side):
    dev = w.chain_device(8)
    eta = 1e-6
    res = leads.lead_self_energy(dev, side, E, eta)
    ref = chain_surface_closed_form(complex(E, eta))
    assert res.converged
    assert abs(res.g_surf[0, 0] - ref) <= 1e-12 * abs(ref)
    # Sigma = t^2 g for the chain
    assert abs(res.sigma_r[0, 0] - ref) <= 1e-12 * abs(ref)
    # retarded: Im Sigma <= 0, i.e. Gamma >= 0
    assert res.gamma[0, 0].real >= -1e-15


def test_chain_iteration_counts():
    dev = w.chain_device(4)
    inb = leads.lead_self_energy(dev, 0, 0.7, 1e-8)
    outb = leads.lead_self_energy(dev, 0, 2.6, 1e-8)
    # doubling: in band the count follows log2(v / eta); out of band it is short
    assert 20 <= inb.iters <= 40
    assert outb.iters <= 10


@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("seed", [11, 12])
def test_decimation_matches_explicit_finite_lead(side, seed):
    """Orientation pin: a 400-cell explicit lead written from the raw blocks."""
    dev = w.random_device(3, 4, seed, overlap=0.05)
    E, eta = 0.35, 0.1
    sr = leads.lead_self_energy(dev, side, E, eta).sigma_r
    bf = dense.explicit_lead_self_energy(dev, side, E, eta, n_cells=400)
    assert np.linalg.norm(sr - bf) <= 1e-11 * np.linalg.norm(bf)


def test_asymmetric_coupling_distinguishes_orientation():
    """The pin above is only a pin if alpha <-> beta gives a different answer."""
    dev = w.random_device(3, 4, 11, overlap=0.05)
    E, eta = 0.35, 0.1
    d, a, b = leads.lead_blocks(dev, 0, E, eta)
    good, _, _ = leads.sancho_rubio(d, a, b)
    swapped, _, _ = leads.sancho_rubio(d, b, a)
    assert np.linalg.norm(a @ good @ b - b @ swapped @ a) > 1e-3 * np.linalg.norm(a @ good @ b)


def test_gamma_psd_and_residual_slab():
    dev = w.slab_device(2, 64, 5)
    for E in (-1.2, 0.1, 0.9):
        for side in (0, 1):
            r = leads.lead_self_energy(dev, side, E, 1e-8)
            assert r.converged
            assert r.residual < 1e-10
            ev = np.linalg.eigvalsh(0.5 * (r.gamma + r.gamma.conj().T))
            assert ev.min() > -1e-9 * max(1.0, ev.max())
            # Gamma is Hermitian by construction
            assert np.linalg.norm(r.gamma - r.gamma.conj().T) <= 1e-13 * max(1.0, np.linalg.norm(r.gamma))


def test_fermi_function():
    assert leads.fermi(0.0, 0.025) == 0.5
    for x in (-0.3, -0.01, 0.02, 0.7, 50.0):
        assert abs(leads.fermi(x, 0.025) + leads.fermi(-x, 0.025) - 1.0) < 1e-15
    assert leads.fermi(-1.0, 0.025) == pytest.approx(1.0 / (1.0 + np.exp(-40.0)), rel=1e-14)


def test_lesser_greater_relation():
    g = np.array([[2.0, 0.5j], [-0.5j, 1.0]])
    sl, sg = leads.lesser_greater(g, 0.3)
    # Sigma^> - Sigma^< = -i Gamma for any occupation
    assert np.allclose(sg - sl, -1j * g, atol=1e-15)
    assert np.allclose(sl, 1j * 0.3 * g)


def _decimate(d, a, c, steps):
    """The decimation state (eps, eps_s, a_k, c_k) after each of `steps` steps."""
    eps_s, eps = d.copy(), d.copy()
    out = []
    for _ in range(steps):
        g = np.linalg.inv(eps)
        agc, cga = a @ g @ c, c @ g @ a
        eps_s, eps = eps_s - agc, eps - agc - cga
        a, c = a @ g @ a, c @ g @ c
        out.append((eps, eps_s, a, c))
    return out


@pytest.mark.parametrize("case", ["random", "slab"])
def test_seeded_closure_exact_for_exact_seed(case):
    """Closing the decimated chain with the exact surface Green's function
    reproduces it after any number of steps (the closure is an identity, not
    an approximation, when the seed is exact)."""
    if case == "random":
        dev, E, eta, tol = w.random_device(3, 3, 13, overlap=0.05), 0.35, 0.05, 1e-12
    else:
        dev, E, eta, tol = w.slab_device(2, 32, 5), 0.1, 1e-8, 1e-9
    d, a, c = leads.lead_blocks(dev, 0, E, eta)
    gs, _, conv = leads.sancho_rubio(d, a, c)
    assert conv
    d_seed = d - a @ gs @ c
    for eps, eps_s, ak, ck in _decimate(d, a, c, 5):
        gk = leads.seeded_closure(eps, eps_s, ak, ck, d_seed)
        assert np.linalg.norm(gk - gs) <= tol * np.linalg.norm(gs)


def test_seeded_closure_tends_to_plain_result():
    """With a useless seed the closure still converges to eps_s^{-1} as the couplings vanish."""
    dev = w.random_device(3, 3, 13, overlap=0.05)
    d, a, c = leads.lead_blocks(dev, 1, 0.35, 0.05)
    gs, it, _ = leads.sancho_rubio(d, a, c)
    eps, eps_s, ak, ck = _decimate(d, a, c, it)[-1]
    gk = leads.seeded_closure(eps, eps_s, ak, ck, d)   # seed 0: d_seed = d
    assert np.linalg.norm(gk - gs) <= 1e-12 * np.linalg.norm(gs)


def test_seeded_decimation_paths():
    dev = w.slab_device(2, 32, 5)
    d, a, c = leads.lead_blocks(dev, 0, 0.1, 1e-8)
    gs, plain_steps, _ = leads.sancho_rubio(d, a, c)
    r = np.random.default_rng(1)
    noise = r.standard_normal(gs.shape) + 1j * r.standard_normal(gs.shape)
    noise *= np.linalg.norm(gs) / np.linalg.norm(noise)
    g, k, how = leads.seeded_sancho_rubio(d, a, c, gs)
    assert how == "candidate" and k == 0
    g, k, how = leads.seeded_sancho_rubio(d, a, c, gs + 1e-6 * noise)
    assert how == "closure" and 0 < k < plain_steps
    assert leads.dyson_residual(d, a, c, g) <= 1e-8
    assert np.linalg.norm(g - gs) <= 1e-6 * np.linalg.norm(gs)
    g, k, how = leads.seeded_sancho_rubio(d, a, c, np.zeros_like(gs))
    assert how in ("closure", "plain") and k <= plain_steps
    assert np.linalg.norm(g - gs) <= 1e-7 * np.linalg.norm(gs)
