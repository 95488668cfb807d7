"""Pins of the self-consistent loop oracle (oracle/scba.py) against what the
physics and the mathematics fix, with no second implementation of the loop:

* no bath: one solve, zero self-energies, the dense brute-force inverse;
* equilibrium (one Fermi level, the bath at the same temperature): every
  iterate obeys the Fermi relation (1 - f) G^< + f G^> = 0 exactly, which
  fixes the direction of the convolution (E - w, not E + w) and the pairing of
  G^< with W^< and G^> with W^>;
* an elastic bath (a single frequency w = 0) conserves the current at every
  energy once converged, and an inelastic one the energy-integrated current,
  at every interface and equal to what the left lead injects -- this fixes the
  retarded self-energy (Sigma^> - Sigma^<) / 2 to its sign and factor;
* the converged self-energies are a fixed point when G^<> is recomputed by
  dense inversion;
* -i Sigma^< and i Sigma^> stay positive semi-definite;
* the fixed point does not depend on the mixing.

Planted mistakes in the oracle's sources must each fail one of these."""
import math
import os
import sys
import types

import numpy as np
import pytest

import workloads as w

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
MODS = ["leads", "dense", "rgf", "observables", "econv", "scba"]
KT = 0.025


def load(tag, target=None, old=None, new=None):
    pkg_name = f"_oracle_scba_variant_{tag}"
    for m in list(sys.modules):
        if m == pkg_name or m.startswith(pkg_name + "."):
            del sys.modules[m]
    pkg = types.ModuleType(pkg_name)
    pkg.__path__ = []
    sys.modules[pkg_name] = pkg
    for name in MODS:
        src = open(os.path.join(ORACLE_DIR, name + ".py")).read()
        if name == target:
            assert old in src, f"mutation anchor not found in {name}: {old!r}"
            src = src.replace(old, new, 1)
        mod = types.ModuleType(f"{pkg_name}.{name}")
        mod.__package__ = pkg_name
        sys.modules[mod.__name__] = mod
        exec(compile(src, f"<{name} variant>", "exec"), mod.__dict__)
        setattr(pkg, name, mod)
    return pkg


def _device():
    return w.folded_chain_device(4, 4)


def _grid(n=48):
    E = w.energy_grid(-1.5, 1.5, n)
    return E, float(E[1] - E[0])


def _coupling(dev, E, i):
    return E * dev.s_upper(i) - dev.H_upper[i]


def _currents(o, dev, pts):
    """[n_e][interfaces] interface currents and [n_e] left-lead injection."""
    j = np.array([o.observables.currents([_coupling(dev, p.E, i) for i in range(dev.nb - 1)], p.GL_upper)
                  for p in pts])
    inj = []
    for p in pts:
        sl, sg = o.leads.lesser_greater(p.lead_l.gamma, p.fl)
        inj.append(o.observables.lead_current(sl, sg, p.GL_diag[0], p.GG_diag[0]))
    return j, np.array(inj)


def pins(o, stop_early=False):
    """{pin: passed} for oracle variant ``o`` (with ``stop_early``, up to the first failure)."""
    ok = {}
    dev = _device()
    E, dE = _grid()
    nb, b = dev.nb, dev.b
    n_w, k0 = 17, 8
    scale = 1j * dE / (2 * math.pi)
    Wl, Wg = w.boson_bath(nb, b, n_w, k0, dE, KT, strength=1.0)

    # no bath: the first solve is the answer, and it is the dense inverse
    Z = np.zeros_like(Wl)
    r = o.scba.scba(dev, E[::6], 1e-6, 0.1, -0.1, KT, Z, Z, k0, scale, tol=1e-12, max_iter=5)
    good = r.n_iter == 1 and r.converged and not np.any(r.sig_l) and not np.any(r.sig_g)
    for p in r.points:
        d = o.dense.solve_point(dev, p.E, 1e-6, 0.1, -0.1, KT)
        Gd, _, _ = o.dense.blocks_of(d["G"], nb, b)
        Ld, _, _ = o.dense.blocks_of(d["Gl"], nb, b)
        good = good and np.allclose(p.GR_diag, Gd, rtol=0, atol=1e-10 * np.abs(Gd).max())
        good = good and np.allclose(p.GL_diag, Ld, rtol=0, atol=1e-10 * np.abs(Ld).max())
    ok["no_bath_is_dense_inverse"] = bool(good)

    if stop_early and not all(ok.values()):
        return ok
    # equilibrium: the Fermi relation at every iterate (three solves, no stopping)
    mu = 0.05
    r = o.scba.scba(dev, E, 1e-6, mu, mu, KT, Wl, Wg, k0, scale, mixing=0.7, tol=0.0, max_iter=3)
    worst = 0.0
    for e, p in enumerate(r.points):
        f = o.leads.fermi(p.E - mu, KT)
        for X, Y in ((p.GL_diag, p.GG_diag), (p.GL_upper, p.GG_upper), (r.sig_l[e], r.sig_g[e])):
            scl = np.abs(X).max() + np.abs(Y).max()
            if scl > 0:
                worst = max(worst, float(np.abs((1 - f) * X + f * Y).max() / scl))
    ok["equilibrium_fermi_relation"] = r.n_iter == 3 and worst < 1e-11 and np.abs(r.sig_l).max() > 1e-4

    if stop_early and not all(ok.values()):
        return ok
    # elastic bath (one frequency, w = 0): current conserved at every energy once converged
    K = np.exp(-np.abs(np.arange(b)[:, None] - np.arange(b)[None, :]) / 2.0)
    We = np.broadcast_to(-1j * 0.05 * K, (1, nb, b, b)).copy()
    r = o.scba.scba(dev, E, 1e-6, 0.1, -0.1, KT, We, We, 0, 1j, mixing=1.0, tol=1e-13, max_iter=60)
    j, inj = _currents(o, dev, r.points)
    jmax = np.abs(j).max()
    ok["elastic_current_per_energy"] = bool(r.converged and jmax > 1e-3
                                            and np.abs(j - j[:, :1]).max() <= 1e-9 * jmax
                                            and np.abs(j[:, 0] - inj).max() <= 1e-9 * jmax)
    # the self-energies stay in the signs of a physical bath
    psd = True
    for e in range(len(E)):
        for i in range(nb):
            sl, sg = r.sig_l[e, i], r.sig_g[e, i]
            psd = psd and np.allclose(sl, -sl.conj().T, atol=1e-14) and np.allclose(sg, -sg.conj().T, atol=1e-14)
            psd = psd and np.linalg.eigvalsh(-1j * sl).min() >= -1e-14 and np.linalg.eigvalsh(1j * sg).min() >= -1e-14
            psd = psd and np.allclose(r.sig_r[e, i], 0.5 * (sg - sl), atol=0)
    ok["self_energy_signs"] = bool(psd)

    if stop_early and not all(ok.values()):
        return ok
    # inelastic bath: the energy-integrated current is the same at every interface and equals the injection
    r = o.scba.scba(dev, E, 1e-6, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=1.0, tol=1e-13, max_iter=60)
    j, inj = _currents(o, dev, r.points)
    J, Jin = j.sum(axis=0), inj.sum()
    spread = float(np.abs(j - j[:, :1]).max() / np.abs(j).max())
    ok["inelastic_integrated_current"] = bool(r.converged and np.abs(J - J[0]).max() <= 1e-9 * abs(J[0])
                                              and abs(J[0] - Jin) <= 1e-9 * abs(J[0]) and spread > 1e-4)
    # and the converged self-energies reproduce themselves through dense inversion
    Gl = np.empty_like(r.sig_l)
    Gg = np.empty_like(r.sig_g)
    for e, p in enumerate(r.points):
        de = w.BTDevice(dev.H_diag, dev.H_upper, dev.S_diag, dev.S_upper, r.sig_r[e], r.sig_l[e], r.sig_g[e])
        d = o.dense.solve_point(de, p.E, 1e-6, 0.1, -0.1, KT)
        Gl[e] = o.dense.blocks_of(d["Gl"], nb, b)[0]
        Gg[e] = o.dense.blocks_of(d["Gg"], nb, b)[0]
    n_e = len(E)
    Fl = o.econv.energy_convolution(Gl.reshape(n_e, -1), Wl.reshape(n_w, -1), k0, scale).reshape(Gl.shape)
    Fg = o.econv.energy_convolution(Gg.reshape(n_e, -1), Wg.reshape(n_w, -1), k0, scale).reshape(Gg.shape)
    num = math.sqrt(np.sum(np.abs(Fl - r.sig_l) ** 2) + np.sum(np.abs(Fg - r.sig_g) ** 2))
    den = math.sqrt(np.sum(np.abs(Fl) ** 2) + np.sum(np.abs(Fg) ** 2))
    ok["fixed_point_by_dense_inversion"] = bool(num <= 1e-10 * den)

    if stop_early and not all(ok.values()):
        return ok
    # a different mixing reaches the same fixed point
    r2 = o.scba.scba(dev, E, 1e-6, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=0.6, tol=1e-13, max_iter=80)
    ok["mixing_independent"] = bool(r2.converged and np.abs(r2.sig_l - r.sig_l).max() <= 1e-10 * np.abs(r.sig_l).max()
                                    and np.abs(r2.sig_g - r.sig_g).max() <= 1e-10 * np.abs(r.sig_g).max())
    return ok


MUTATIONS = [
    ("scba", "return 0.5 * (sig_g - sig_l)", "return sig_g - sig_l"),
    ("scba", "return 0.5 * (sig_g - sig_l)", "return 0.5 * (sig_l - sig_g)"),
    ("scba", "W_g.reshape(n_w, -1), k0, scale)", "W_l.reshape(n_w, -1), k0, scale)"),
    ("scba", "sig_l=sig_l[e], sig_g=sig_g[e]", "sig_l=sig_g[e], sig_g=sig_l[e]"),
    ("scba", "Sg = Sg + mixing * (Fg - Sg)", "Sg = Sg + mixing * (Fl - Sg)"),
    ("scba", "return math.sqrt(num / den)", "return 1e-3 * math.sqrt(num / den)"),
    ("econv", "shift = k0 - k ", "shift = k - k0 "),
]


def test_unmutated_scba_oracle_passes_every_pin():
    res = pins(load("clean"))
    assert all(res.values()), res


@pytest.mark.parametrize("k", range(len(MUTATIONS)))
def test_planted_mistake_in_the_loop_is_caught(k):
    target, old, new = MUTATIONS[k]
    with np.errstate(all="ignore"):
        try:
            res = pins(load(f"m{k}", target, old, new), stop_early=True)
        except (np.linalg.LinAlgError, ValueError, FloatingPointError):
            return
    assert not all(res.values()), f"mutation {k} ({target}: {new!r}) passed every pin: {res}"


def test_boson_bath_detailed_balance_and_symmetry():
    """The bath the loop tests use: W^>(w) = e^{w/kT} W^<(w), W^<(w) = W^>(-w) on a symmetric grid,
    i W^<> positive semi-definite in every block (the spatial kernel is positive definite)."""
    nb_, b, n_w, k0, dE = 2, 6, 21, 10, 0.03
    Wl, Wg = w.boson_bath(nb_, b, n_w, k0, dE, KT, strength=0.7)
    for k in range(n_w):
        om = (k - k0) * dE
        assert np.allclose(Wg[k], np.exp(om / KT) * Wl[k], rtol=1e-12, atol=0), k
        assert np.allclose(Wl[k], Wg[2 * k0 - k], rtol=1e-12, atol=1e-300), k
        for blk in range(nb_):
            for X in (Wl[k, blk], Wg[k, blk]):
                assert np.allclose(X, X.T)
                assert np.linalg.eigvalsh((1j * X).real).min() >= -1e-14


def test_k_points_average_and_conserve_the_summed_current():
    """Several k-points: identical devices at every k give the single-device loop exactly; two
    different k-devices, converged, conserve the energy-integrated current summed over k at every
    interface (the pairing argument of the single-device pin applies to the k-averaged G^<>)."""
    from oracle import scba, observables
    dev = w.folded_chain_device(4, 4)
    E, dE = _grid(32)
    n_w, k0 = 9, 4
    scale = 1j * dE / (2 * math.pi)
    Wl, Wg = w.boson_bath(dev.nb, dev.b, n_w, k0, dE, KT, strength=1.0)
    one = scba.scba(dev, E, 1e-6, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=1.0, tol=0.0, max_iter=3)
    two = scba.scba([dev, dev], E, 1e-6, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=1.0, tol=0.0, max_iter=3)
    assert np.array_equal(one.sig_l, two.sig_l) and np.array_equal(one.sig_g, two.sig_g)
    # two genuinely different k-points of a wire with transverse hopping
    base = w.folded_chain_device(4, 4)
    T = 0.2 * np.eye(4, k=1)
    devs = []
    for kk in (0.0, 1.3):
        ph = complex(math.cos(kk), math.sin(kk))
        H = np.stack([h + ph * T + np.conj(ph) * T.T for h in base.H_diag])
        devs.append(w.BTDevice(H, base.H_upper))
    r = scba.scba(devs, E, 1e-6, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=1.0, tol=1e-13, max_iter=60)
    assert r.converged
    J = np.zeros(base.nb - 1)
    for d, pk in zip(devs, r.points):
        for p in pk:
            J += observables.currents([p.E * d.s_upper(i) - d.H_upper[i] for i in range(d.nb - 1)], p.GL_upper)
    assert np.abs(J - J[0]).max() <= 1e-9 * abs(J[0]), J


def test_anderson_mixing_reaches_the_fixed_point_where_linear_mixing_does_not():
    """Anderson's extrapolation (memory 3): on a contractive case the same fixed point as linear mixing
    (1e-10) in fewer solves; on a periodic wire at a coupling where linear mixing first converges and then
    diverges (an unstable mode grows out of rounding), it converges; memory 0 is linear mixing exactly."""
    from oracle import scba
    dev = w.folded_chain_device(4, 4)
    E, dE = _grid(32)
    n_w, k0 = 9, 4
    scale = 1j * dE / (2 * math.pi)
    Wl, Wg = w.boson_bath(dev.nb, dev.b, n_w, k0, dE, KT, strength=1.0)
    lin = scba.scba(dev, E, 1e-6, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=0.5, tol=1e-12, max_iter=80)
    and3 = scba.scba(dev, E, 1e-6, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=0.5, tol=1e-12, max_iter=80, memory=3)
    assert lin.converged and and3.converged and and3.n_iter < lin.n_iter, (lin.n_iter, and3.n_iter)
    assert np.abs(and3.sig_l - lin.sig_l).max() <= 1e-10 * np.abs(lin.sig_l).max()
    zero = scba.scba(dev, E, 1e-6, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=0.5, tol=0.0, max_iter=4, memory=0)
    ref = scba.scba(dev, E, 1e-6, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=0.5, tol=0.0, max_iter=4)
    assert np.array_equal(zero.sig_l, ref.sig_l)
    wire = w.periodic_wire_device(4, 4, 3)
    Ew = w.energy_grid(-3.0, 3.0, 64)
    dEw = float(Ew[1] - Ew[0])
    Wl, Wg = w.boson_bath(wire.nb, wire.b, 17, 8, dEw, KT, strength=0.2)
    sw = 1j * dEw / (2 * math.pi)
    lin = scba.scba(wire, Ew, 1e-6, 0.1, -0.1, KT, Wl, Wg, 8, sw, mixing=1.0, tol=1e-12, max_iter=40)
    assert not lin.converged and lin.history[-1] > 1e-9
    acc = scba.scba(wire, Ew, 1e-6, 0.1, -0.1, KT, Wl, Wg, 8, sw, mixing=1.0, tol=1e-12, max_iter=40, memory=3)
    assert acc.converged, acc.history


def test_anderson_step_solves_a_linear_fixed_point_like_gmres():
    """On a linear map x -> G x + c of dimension d, Anderson's extrapolation with memory >= d and mixing 1
    is equivalent to GMRES on (I - G) x = c (Walker and Ni, SIAM J. Numer. Anal. 49, 1715 (2011)): it
    reaches the exact solution within d + 1 updates, also where plain iteration diverges (eigenvalues of G
    outside the unit disc).  A dropped difference, a wrong sign of gamma or a transposed normal matrix
    fails this."""
    from oracle.scba import anderson
    rng = np.random.default_rng(7)
    d = 4
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    G = Q @ np.diag([1.7, -2.5, 0.4, 0.9]) @ Q.T          # spectral radius 2.5: plain iteration diverges
    c = rng.standard_normal(d)
    exact = np.linalg.solve(np.eye(d) - G, c)
    for memory in (d, d + 2):
        x, prev, dxs, dfs = np.zeros(d), None, [], []
        errs = []
        for n in range(d + 2):
            f = G @ x + c - x
            if prev is not None:
                dxs.append(x - prev[0])
                dfs.append(f - prev[1])
                dxs, dfs = dxs[-memory:], dfs[-memory:]
            prev = (x, f)
            x = anderson(x, f, dxs, dfs, 1.0)
            errs.append(float(np.linalg.norm(x - exact) / np.linalg.norm(exact)))
        assert errs[d] < 1e-9, (memory, errs)
    # plain iteration from the same start runs away
    x = np.zeros(d)
    for _ in range(d + 2):
        x = G @ x + c
    assert np.linalg.norm(x - exact) > np.linalg.norm(exact)
