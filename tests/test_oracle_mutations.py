"""Planted mistakes in the oracle must be caught by its pins.

Each case below edits one line of an oracle module's source text (a dropped
term, a wrong sign, a swapped or transposed operand), loads the edited
modules as a throw-away package on the CPU, and runs the same closed-form,
brute-force and invariant checks that pin the real oracle.  At least one of
them has to fail.  The unedited sources must pass all of them.
"""
import cmath
import os
import sys
import types

import numpy as np
import pytest

import workloads as w

ORACLE_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle")
MODS = ["leads", "dense", "rgf", "observables"]


def load_variant(tag, target=None, old=None, new=None):
    pkg_name = f"_oracle_variant_{tag}"
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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _chain_root(z):
    s = cmath.sqrt(z * z - 4)
    r1, r2 = (z + s) / 2, (z - s) / 2
    return r1 if abs(r1) < 1 else r2


def pins(o):
    """Run the pin checks on oracle variant ``o``; returns {name: passed}."""
    out = {}
    # closed-form chain surface Green's function, both sides
    dev = w.chain_device(6)
    ok = True
    for side in (0, 1):
        for E in (-0.8, 1.3):
            r = o.leads.lead_self_energy(dev, side, E, 1e-6)
            ref = _chain_root(complex(E, 1e-6))
            ok &= abs(r.g_surf[0, 0] - ref) < 1e-10 and r.gamma[0, 0].real >= 0
    out["chain_gs"] = bool(ok)
    # explicit finite lead (orientation)
    dev = w.random_device(3, 3, 11, overlap=0.05)
    ok = True
    for side in (0, 1):
        sr = o.leads.lead_self_energy(dev, side, 0.35, 0.1).sigma_r
        bf = o.dense.explicit_lead_self_energy(dev, side, 0.35, 0.1, n_cells=300)
        ok &= rel(sr, bf) < 1e-10
    out["finite_lead"] = bool(ok)
    # chain transmission through RGF and dense
    dev = w.chain_device(8)
    r = o.rgf.solve_point(dev, 0.6, 1e-6, want_T=True, lesser_greater=False)
    d = o.dense.solve_point(dev, 0.6, 1e-6)
    out["chain_T"] = bool(abs(r.T - 1) < 1e-8 and abs(d["T"] - 1) < 1e-8)
    # ballistic current conservation + Landauer (dense and RGF)
    dev = w.random_device(5, 3, 5, overlap=0.05)
    E = 0.2
    d = o.dense.solve_point(dev, E, 1e-8, 0.1, -0.1, 0.025)
    Ad, Au, Al = o.rgf.assemble_blocks(dev, E, d["lead_l"].sigma_r, d["lead_r"].sigma_r)
    _, Lu, _ = o.dense.blocks_of(d["Gl"], 5, 3)
    land = (d["fl"] - d["fr"]) * d["T"]
    jd = o.observables.currents(Au, Lu)
    r = o.rgf.solve_point(dev, E, 1e-8, 0.1, -0.1, 0.025, want_T=True)
    jr = o.observables.currents(Au, r.GL_upper)
    out["current"] = bool(abs(land) > 1e-6 and np.max(np.abs(jd - land)) < 1e-10 and np.max(np.abs(jr - land)) < 1e-10)
    # scattering identities on dense and RGF vs dense
    dev = w.random_device(4, 3, 21, overlap=0.05)
    w.scattering_self_energies(dev, 3, norm=0.05)
    d = o.dense.solve_point(dev, -0.3, 1e-8, 0.1, -0.1, 0.025)
    G, Gl, Gg = d["G"], d["Gl"], d["Gg"]
    out["I4_I5"] = bool(rel(G - G.conj().T, Gg - Gl) < 1e-11
                        and np.linalg.norm(Gl + Gl.conj().T) < 1e-11 * np.linalg.norm(Gl)
                        and np.linalg.eigvalsh(-1j * 0.5 * (Gl - Gl.conj().T)).min() > -1e-12)
    r = o.rgf.solve_point(dev, -0.3, 1e-8, 0.1, -0.1, 0.025, greater=True, want_T=True)
    Gd, Gu, Glo = o.dense.blocks_of(G, 4, 3)
    Ld, Lu2, _ = o.dense.blocks_of(Gl, 4, 3)
    Hd, Hu, _ = o.dense.blocks_of(Gg, 4, 3)
    out["rgf_vs_dense"] = bool(max(rel(r.GR_diag, Gd), rel(r.GR_upper, Gu), rel(r.GR_lower, Glo),
                                   rel(r.GL_diag, Ld), rel(r.GL_upper, Lu2), rel(r.GG_diag, Hd),
                                   rel(r.GG_upper, Hu)) < 1e-10 and abs(r.T - d["T_rl"]) < 1e-10)
    # seeded closure: exact at every step for the exact seed; a perturbed seed is
    # taken by the closure before the plain decimation would stop
    dev = w.random_device(3, 3, 13, overlap=0.05)
    d_, a_, c_ = o.leads.lead_blocks(dev, 0, 0.35, 0.05)
    gs, steps, _ = o.leads.sancho_rubio(d_, a_, c_)
    ok = True
    eps_s, eps, ak, ck = d_.copy(), d_.copy(), a_.copy(), c_.copy()
    d_seed = d_ - a_ @ gs @ c_
    for _ in range(4):
        g = np.linalg.inv(eps)
        agc, cga = ak @ g @ ck, ck @ g @ ak
        eps_s, eps = eps_s - agc, eps - agc - cga
        ak, ck = ak @ g @ ak, ck @ g @ ck
        ok &= rel(o.leads.seeded_closure(eps, eps_s, ak, ck, d_seed), gs) < 1e-10
    g, k, how = o.leads.seeded_sancho_rubio(d_, a_, c_, gs)
    ok &= how == "candidate" and k == 0 and rel(g, gs) < 1e-12
    noise = np.random.default_rng(2).standard_normal(gs.shape) * np.linalg.norm(gs) / 3.0
    g, k, how = o.leads.seeded_sancho_rubio(d_, a_, c_, gs + 1e-6 * noise)
    ok &= how == "closure" and k < steps and rel(g, gs) < 1e-6
    out["seeded_closure"] = bool(ok)
    # density of states of a chain segment: the bulk closed form at every site
    r = o.rgf.solve_point(w.chain_device(8), 0.45, 1e-9, lesser_greater=False)
    ref = 1.0 / (np.pi * np.sqrt(4.0 - 0.45 ** 2))
    out["chain_dos"] = bool(np.max(np.abs(o.observables.dos(r.GR_diag) - ref)) < 1e-6 * ref)
    return out


MUTATIONS = [
    ("rgf", "Gd[i] = g[i] - X[i] @ Gl[i]", "Gd[i] = g[i] + X[i] @ Gl[i]"),
    ("rgf", "Gl[i] = -Gd[i + 1] @ Al[i] @ g[i]", "Gl[i] = -Gd[i + 1] @ Au[i] @ g[i]"),
    ("rgf", "X[i - 1] = g[i - 1] @ Au[i - 1]", "X[i - 1] = Au[i - 1] @ g[i - 1]"),
    ("rgf", "Gu[i] = -X[i] @ Gd[i + 1]", "Gu[i] = -Gd[i + 1] @ X[i]"),
    ("rgf", "Ld[i] = gl[i] + Z @ X[i].conj().T + Q - Q.conj().T", "Ld[i] = gl[i] + Z @ X[i].conj().T + Q"),
    ("rgf", "Lu[i] = V.conj().T @ Gd[i + 1].conj().T - Z", "Lu[i] = V.conj().T @ Gd[i + 1].conj().T + Z"),
    ("rgf", "Z = X[i] @ Ld[i + 1]", "Z = X[i] @ Ld[i + 1].T"),
    ("rgf", "Bt = sig_diag[i] + Al[i - 1] @ gl[i - 1] @ Al[i - 1].conj().T",
     "Bt = Al[i - 1] @ gl[i - 1] @ Al[i - 1].conj().T"),
    ("rgf", "C = -g[i] @ Al[i - 1] @ C", "C = -g[i] @ Al[i - 1].T @ C"),
    ("rgf", "np.trace(gamma_r @ C @ gamma_l @ C.conj().T)", "np.trace(gamma_l @ C @ gamma_r @ C.conj().T)"),
    ("rgf", "Al = [u.conj().T for u in Au]", "Al = [u.T for u in Au]"),
    ("rgf", "a = E * dev.s_diag(i) - dev.H_diag[i]", "a = E * dev.s_diag(i) + dev.H_diag[i]"),
    ("leads", "alpha = H1 - z * S1", "alpha = H1.conj().T - z * S1.conj().T"),
    ("leads", "beta = H1.conj().T - z * S1.conj().T", "beta = H1 - z * S1"),
    ("leads", "eps = eps - agc - cga", "eps = eps - agc"),
    ("leads", "c = c @ g @ c", "c = c @ g @ a"),
    ("leads", "z = complex(E, eta)", "z = complex(E, -eta)"),
    ("leads", "gam = 1j * (sig - sig.conj().T)", "gam = 1j * (sig - sig.T)"),
    ("leads", "return 1j * f * gamma, -1j * (1.0 - f) * gamma", "return 1j * f * gamma, -1j * f * gamma"),
    ("leads", "H1, S1 = dev.H_upper[0].conj().T, dev.s_upper(0).conj().T", "H1, S1 = dev.H_upper[0], dev.s_upper(0)"),
    ("leads", "X = np.linalg.inv(eps - eps_s + d_seed)", "X = np.linalg.inv(eps + d_seed)"),
    ("leads", "return np.linalg.inv(eps_s - a @ X @ c)", "return np.linalg.inv(eps_s - c @ X @ a)"),
    ("leads", "d_seed = d - alpha @ g_seed @ beta", "d_seed = d - beta @ g_seed @ alpha"),
    ("dense", "A[s1, s0] = up.conj().T", "A[s1, s0] = up.T"),
    ("dense", "Gl = G @ Sl @ GH", "Gl = GH @ Sl @ G"),
    ("dense", "A[N - b:, N - b:] -= sig_right", "A[N - b:, N - b:] += sig_right"),
    ("dense", "Sg[sl, sl] += dev.sig_g[i]", "Sg[sl, sl] += dev.sig_l[i]"),
    ("observables", "return float(-2.0 * np.real(np.trace(A_upper @ GL_lower)))",
     "return float(-2.0 * np.imag(np.trace(A_upper @ GL_lower)))"),
    ("observables", "-np.imag(np.trace(g)) / np.pi", "-np.imag(np.trace(g)) / (2 * np.pi)"),
    ("observables", "-np.imag(np.trace(g)) / np.pi", "np.imag(np.trace(g)) / np.pi"),
]


def test_unmutated_oracle_passes_every_pin():
    res = pins(load_variant("clean"))
    assert all(res.values()), res


@pytest.mark.parametrize("k", range(len(MUTATIONS)))
def test_planted_mistake_is_caught(k):
    target, old, new = MUTATIONS[k]
    with np.errstate(all="ignore"):
        try:
            res = pins(load_variant(f"m{k}", target, old, new))
        except (np.linalg.LinAlgError, ValueError, FloatingPointError):
            return  # the mistake breaks the computation outright
    assert not all(res.values()), f"mutation {k} ({target}: {new!r}) passed every pin: {res}"
