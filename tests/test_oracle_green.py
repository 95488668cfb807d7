"""Pins of the dense and RGF oracles: closed forms, invariants and brute force."""
import cmath

import numpy as np
import pytest

import workloads as w
from oracle import dense, leads, observables, rgf


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("E", [-1.9, -1.3, -0.55, 0.25, 0.8, 1.6])
def test_chain_transmission_in_band_is_one(E):
    dev = w.chain_device(32)
    d = dense.solve_point(dev, E, 1e-6)
    r = rgf.solve_point(dev, E, 1e-6, want_T=True, lesser_greater=False)
    assert abs(d["T"] - 1.0) < 1e-9
    assert abs(r.T - 1.0) < 1e-9


@pytest.mark.parametrize("E", [-2.9, -2.3, 2.2, 2.8])
def test_chain_transmission_out_of_band_is_zero(E):
    dev = w.chain_device(32)
    r = rgf.solve_point(dev, E, 1e-6, want_T=True, lesser_greater=False)
    assert abs(r.T) < 1e-12


@pytest.mark.parametrize("E", [-1.5, -0.4, 0.7, 2.4])
def test_chain_diagonal_equals_infinite_chain(E):
    """G_00 of the chain between two leads is the infinite-chain 1/sqrt((E-eps)^2 - 4t^2)."""
    dev = w.chain_device(32)
    eta = 1e-6
    r = rgf.solve_point(dev, E, eta, lesser_greater=False)
    s = cmath.sqrt(E * E - 4.0)
    ref = 1.0 / s
    if ref.imag > 0:
        ref = -ref
    if abs(E) > 2:
        ref = np.sign(E) / np.sqrt(E * E - 4.0)
    for i in (0, 15, 31):
        assert abs(r.GR_diag[i, 0, 0] - ref) < 1e-5


@pytest.mark.parametrize("E", [-1.3, 0.45, 1.2])
def test_folded_chain_transmission_is_one(E):
    dev = w.folded_chain_device(6, 8)
    r = rgf.solve_point(dev, E, 1e-6, want_T=True, lesser_greater=False)
    assert abs(r.T - 1.0) < 1e-8


def test_periodic_wire_transmission_is_integer():
    dev = w.periodic_wire_device(6, 8, seed=7)
    Ts = []
    for E in np.linspace(-2.0, 2.0, 23):
        r = rgf.solve_point(dev, E, 1e-6, want_T=True, lesser_greater=False)
        Ts.append(r.T)
    Ts = np.array(Ts)
    assert np.max(np.abs(Ts - np.round(Ts))) < 1e-5
    assert Ts.max() >= 2.0 - 1e-5          # several open channels somewhere in the range


# ---------------------------------------------------------------- invariants

def _ballistic(seed=5, nb=6, b=4, E=0.2):
    dev = w.random_device(nb, b, seed, overlap=0.05)
    d = dense.solve_point(dev, E, 1e-8, 0.1, -0.1, 0.025)
    return dev, d


def test_current_conservation_and_landauer():
    dev, d = _ballistic()
    nb, b = dev.nb, dev.b
    E = 0.2
    Ad, Au, Al = rgf.assemble_blocks(dev, E, d["lead_l"].sigma_r, d["lead_r"].sigma_r)
    _, Lu, _ = dense.blocks_of(d["Gl"], nb, b)
    j = observables.currents(Au, Lu)
    landauer = (d["fl"] - d["fr"]) * d["T"]
    assert abs(landauer) > 1e-6
    assert np.max(np.abs(j - landauer)) < 1e-10 * max(1.0, abs(landauer)) + 1e-13
    sl, sg = leads.lesser_greater(d["lead_l"].gamma, d["fl"])
    Gl00 = d["Gl"][:b, :b]
    Gg00 = d["Gg"][:b, :b]
    assert abs(observables.lead_current(sl, sg, Gl00, Gg00) - landauer) < 1e-12


def test_transmission_reciprocity():
    _, d = _ballistic(seed=8)
    assert abs(d["T_lr"] - d["T_rl"]) < 1e-12 * max(1.0, d["T_lr"])


def test_single_block_transmission_formula():
    """T = Tr[Gamma_L (i(G00 - G00^H) - G00 Gamma_L G00^H)] in the ballistic limit."""
    dev, d = _ballistic(seed=9)
    b = dev.b
    G00 = d["G"][:b, :b]
    gl = d["lead_l"].gamma
    t1 = np.real(np.trace(gl @ (1j * (G00 - G00.conj().T) - G00 @ gl @ G00.conj().T)))
    assert abs(t1 - d["T"]) < 1e-10


def test_scattering_identities_dense():
    dev = w.random_device(5, 4, 21, overlap=0.05)
    w.scattering_self_energies(dev, 3, norm=0.05)
    d = dense.solve_point(dev, -0.3, 1e-8, 0.1, -0.1, 0.025)
    G, Gl, Gg = d["G"], d["Gl"], d["Gg"]
    # I4: G^R - G^A = G^> - G^<
    assert rel(G - G.conj().T, Gg - Gl) < 1e-12
    # I5: anti-Hermitian lesser, -iG^< and iG^> PSD
    assert np.linalg.norm(Gl + Gl.conj().T) < 1e-12 * np.linalg.norm(Gl)
    assert np.linalg.eigvalsh(-1j * Gl).min() > -1e-12
    assert np.linalg.eigvalsh(1j * Gg).min() > -1e-12
    # I3 block rows: (A G^<)_ii = Sigma^<_ii (G_ii)^H (global identity A G^< = Sigma^< G^A)
    b = dev.b
    AGl = d["A"] @ Gl
    sl_l = leads.lesser_greater(d["lead_l"].gamma, d["fl"])[0] + dev.sig_l[0]
    assert rel(AGl[:b, :b], sl_l @ G[:b, :b].conj().T) < 1e-11


# ---------------------------------------------------------------- RGF vs brute force

@pytest.mark.parametrize("seed,nb,b,E", [(1, 6, 4, 0.3), (2, 5, 7, -0.6), (3, 2, 5, 1.1), (4, 9, 3, 0.05)])
@pytest.mark.parametrize("scatter", [False, True])
def test_rgf_matches_dense(seed, nb, b, E, scatter):
    dev = w.random_device(nb, b, seed, overlap=0.05)
    if scatter:
        w.scattering_self_energies(dev, seed + 100, norm=0.05)
    r = rgf.solve_point(dev, E, 1e-8, 0.1, -0.1, 0.025, greater=True, want_T=True)
    d = dense.solve_point(dev, E, 1e-8, 0.1, -0.1, 0.025)
    Gd, Gu, Gl = dense.blocks_of(d["G"], nb, b)
    Ld, Lu, _ = dense.blocks_of(d["Gl"], nb, b)
    Hd, Hu, _ = dense.blocks_of(d["Gg"], nb, b)
    assert rel(r.GR_diag, Gd) < 1e-12
    assert rel(r.GR_upper, Gu) < 1e-12
    assert rel(r.GR_lower, Gl) < 1e-12
    assert rel(r.GL_diag, Ld) < 1e-11
    assert rel(r.GL_upper, Lu) < 1e-11
    assert rel(r.GG_diag, Hd) < 1e-11
    assert rel(r.GG_upper, Hu) < 1e-11
    assert abs(r.T - d["T_rl"]) < 1e-11 * max(1.0, abs(d["T_rl"])) + 1e-14


def test_rgf_matches_dense_small_workload():
    """The small ballistic workload (Nb=32, b=8, S=I, N=256) at a few energies."""
    dev = w.random_device(32, 8, 1)
    for E in w.energy_grid(-3, 3, 64)[::13]:
        r = rgf.solve_point(dev, E, 1e-6, want_T=True, lesser_greater=False)
        d = dense.solve_point(dev, E, 1e-6)
        Gd, _, _ = dense.blocks_of(d["G"], 32, 8)
        # the two solvers round differently; agreement is set by cond(A) ~ 1e4 here
        assert rel(r.GR_diag, Gd) < 1e-10
        assert abs(r.T - d["T_rl"]) < 1e-10


def test_rgf_matches_dense_slab():
    """A slab-shaped device (sparse blocks, S != I) with scattering, N = 6 * 96."""
    dev = w.slab_device(6, 96, 2)
    w.scattering_self_energies(dev, 3)
    E = 0.37
    r = rgf.solve_point(dev, E, 1e-8, 0.1, -0.1, 0.025, greater=True)
    d = dense.solve_point(dev, E, 1e-8, 0.1, -0.1, 0.025)
    Gd, Gu, Gl = dense.blocks_of(d["G"], 6, 96)
    Ld, Lu, _ = dense.blocks_of(d["Gl"], 6, 96)
    Hd, Hu, _ = dense.blocks_of(d["Gg"], 6, 96)
    assert rel(r.GR_diag, Gd) < 1e-11 and rel(r.GR_upper, Gu) < 1e-11 and rel(r.GR_lower, Gl) < 1e-11
    assert rel(r.GL_diag, Ld) < 1e-10 and rel(r.GL_upper, Lu) < 1e-10
    assert rel(r.GG_diag, Hd) < 1e-10 and rel(r.GG_upper, Hu) < 1e-10


def test_rgf_band_identities():
    """I1/I2: (A G)_ii = I and the local identities of the backward step."""
    dev = w.random_device(7, 5, 31, overlap=0.05)
    E = -0.45
    L = leads.lead_self_energy(dev, 0, E, 1e-8)
    R = leads.lead_self_energy(dev, 1, E, 1e-8)
    Ad, Au, Al = rgf.assemble_blocks(dev, E, L.sigma_r, R.sigma_r)
    g, X, Gd, Gu, Gl = rgf.retarded(Ad, Au, Al)
    eye = np.eye(5)
    nb = 7
    for i in range(nb):
        row = Ad[i] @ Gd[i]
        if i > 0:
            row = row + Al[i - 1] @ Gu[i - 1]
        if i < nb - 1:
            row = row + Au[i] @ Gl[i]
        assert np.linalg.norm(row - eye) < 1e-12
    for i in range(nb - 1):
        M = Ad[i] if i == 0 else Ad[i] - Al[i - 1] @ X[i - 1]
        assert np.linalg.norm(M @ Gd[i] + Au[i] @ Gl[i] - eye) < 1e-12
        assert np.linalg.norm(Gl[i] @ M + Gd[i + 1] @ Al[i]) < 1e-12


def test_dos_positive():
    dev = w.random_device(6, 4, 3)
    r = rgf.solve_point(dev, 0.1, 1e-6, lesser_greater=False)
    assert np.all(observables.dos(r.GR_diag) > 0)


@pytest.mark.parametrize("E", [-1.7, -0.6, 0.3, 1.1, 1.9])
@pytest.mark.parametrize("t", [1.0, 0.7])
def test_dos_chain_closed_form(E, t):
    """Every site of a device cut from an infinite 1D chain (leads repeat it)
    carries the bulk density of states 1 / (pi sqrt(4 t^2 - (E - eps)^2)) inside
    the band (one state per site: the scale is fixed), and the folded chain
    (8 sites per block) carries 8 times it per block."""
    if abs(E) >= 2 * t:
        pytest.skip("outside the band")
    ref = 1.0 / (np.pi * np.sqrt(4 * t * t - E * E))
    r = rgf.solve_point(w.chain_device(12, t=t), E, 1e-9, lesser_greater=False)
    d = observables.dos(r.GR_diag)
    assert np.max(np.abs(d - ref)) < 1e-6 * ref
    rf = rgf.solve_point(w.folded_chain_device(4, 8, t=t), E, 1e-9, lesser_greater=False)
    assert np.max(np.abs(observables.dos(rf.GR_diag) - 8 * ref)) < 1e-6 * 8 * ref
    # outside the band no state is available
    ro = rgf.solve_point(w.chain_device(6, t=t), 2.5 * t, 1e-9, lesser_greater=False)
    assert np.max(np.abs(observables.dos(ro.GR_diag))) < 1e-6
