"""GPU self-consistent loop (negf_scba) and energy-dependent scattering
self-energies (negf_problem.sc_stride) against the oracle (oracle/scba.py,
oracle/rgf.py), plus properties of the loop's output that hold at any size
(the Fermi relation at equilibrium, current conservation once converged)."""
import dataclasses
import math

import numpy as np
import pytest

import workloads as w
from helpers import point_tolerance, record, refined_inversions
from oracle import leads as oleads
from oracle import observables as oobs
from oracle import rgf as orgf
from oracle import scba as oscba

pytestmark = pytest.mark.gpu

KT = 0.025
ETA = 1e-6


@pytest.fixture(scope="module")
def nb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2602_03438_amd import binding
    binding.lib()
    return binding


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _bath(dev, n_e, lo=-1.5, hi=1.5, n_w=17, strength=1.0):
    E = w.energy_grid(lo, hi, n_e)
    dE = float(E[1] - E[0])
    k0 = (n_w - 1) // 2
    Wl, Wg = w.boson_bath(dev.nb, dev.b, n_w, k0, dE, KT, strength=strength)
    return E, dE, k0, Wl, Wg


def _gpu_loop(nb, dev, E, Wl, Wg, k0, scale, mu_l, mu_r, **kw):
    import torch
    prob = nb.Problem(nb.DeviceOnGPU(dev), E, eta=ETA, mu_l=mu_l, mu_r=mu_r, kT=KT)
    print(f"  negf_scba nb={dev.nb} b={dev.b} n_e={len(E)} n_w={Wl.shape[0]} {kw}", flush=True)
    res = nb.scba(prob, torch.from_numpy(Wl).cuda(), torch.from_numpy(Wg).cuda(), k0, scale, **kw)
    torch.cuda.synchronize()
    return res


def _stack(points, name):
    return np.stack([getattr(p, name) for p in points])


# --------------------------------------------------------------- energy-dependent self-energies

@pytest.mark.parametrize("prec,bar", [(0, 1e-10), (1, 1e-6)])
def test_energy_dependent_self_energies_match_oracle(nb, prec, bar):
    """sc_stride = nb b b: energy e of the problem reads its own Sigma_sc; chunked (batch 4 of 6 energies,
    so the second chunk starts inside the problem) and at a block size with a ragged tile (b = 40)."""
    import torch
    base = w.slab_device(5, 40, 2)
    E = np.linspace(-0.9, 1.1, 6)
    per_e = [w.scattering_self_energies(dataclasses.replace(base), 50 + e, norm=0.02) for e in range(E.size)]
    dev = dataclasses.replace(base, sig_r=np.stack([d.sig_r for d in per_e]), sig_l=np.stack([d.sig_l for d in per_e]),
                              sig_g=np.stack([d.sig_g for d in per_e]))
    prob = nb.Problem(nb.DeviceOnGPU(dev), E, eta=ETA, mu_l=0.1, mu_r=-0.1, kT=KT, sc_stride=5 * 40 * 40)
    out = nb.rgf_lesser_greater([prob], prec=prec, opts=nb.make_options(batch=4), greater=True)
    torch.cuda.synchronize()
    assert int(out["info"].abs().sum()) == 0
    names = ("GR_diag", "GR_upper", "GL_diag", "GL_upper", "GG_diag")
    for k, e in enumerate(E):
        ref, tol = point_tolerance(lambda: orgf.solve_point(per_e[k], e, ETA, 0.1, -0.1, KT, greater=True), names,
                                   base=bar)
        for n in names:
            err = rel(out[n][0][k].cpu().numpy(), getattr(ref, n))
            record("energy_dependent_sigma", e, n, err, tol[n], prec=prec)
            assert err < tol[n], (k, n, err, tol[n])


def test_energy_dependent_self_energies_partitioned(nb):
    """The partitioned inversion reads the per-energy self-energies as the sweeps do."""
    import torch
    base = w.slab_device(8, 24, 3)
    E = np.linspace(-0.7, 0.9, 3)
    per_e = [w.scattering_self_energies(dataclasses.replace(base), 70 + e, norm=0.02) for e in range(E.size)]
    dev = dataclasses.replace(base, sig_r=np.stack([d.sig_r for d in per_e]), sig_l=np.stack([d.sig_l for d in per_e]),
                              sig_g=np.stack([d.sig_g for d in per_e]))
    prob = nb.Problem(nb.DeviceOnGPU(dev), E, eta=ETA, mu_l=0.1, mu_r=-0.1, kT=KT, sc_stride=8 * 24 * 24)
    out = nb.serinv_lesser_greater(prob, 2, greater=True)
    torch.cuda.synchronize()
    assert int(out["info"].abs().sum()) == 0
    names = ("GR_diag", "GL_diag", "GG_upper")
    for k, e in enumerate(E):
        ref, tol = point_tolerance(lambda: orgf.solve_point(per_e[k], e, ETA, 0.1, -0.1, KT, greater=True), names)
        for n in names:
            err = rel(out[n][0][k].cpu().numpy(), getattr(ref, n))
            record("energy_dependent_sigma_partitioned", e, n, err, tol[n])
            assert err < tol[n], (k, n, err, tol[n])


# --------------------------------------------------------------- the loop against the oracle

def _loop_reference(compute):
    """(oracle result, {output: spread}) where the spread is how far the whole loop's outputs move
    when every inversion inside it is Newton-refined (its sensitivity to rounding)."""
    ref = compute()
    with refined_inversions():
        ref2 = compute()
    out = {}
    for n in ("sig_l", "sig_g"):
        out[n] = rel(getattr(ref2, n), getattr(ref, n))
    for n in ("GR_diag", "GR_upper", "GL_diag", "GL_upper", "GG_diag"):
        out[n] = rel(_stack(ref2.points, n), _stack(ref.points, n))
    return ref, out


def _compare_loop(test, res, ref, spread, bar=1e-10):
    for n in ("sig_l", "sig_g", "sig_r"):
        got = res[n].cpu().numpy()
        tol = max(bar, 4.0 * spread.get(n, spread["sig_l"]))
        err = rel(got, getattr(ref, n))
        record(test, 0.0, n, err, tol, spread=spread.get(n, spread["sig_l"]))
        assert err < tol, (n, err, tol)
    for n in ("GR_diag", "GR_upper", "GL_diag", "GL_upper", "GG_diag"):
        got = res[n][0].cpu().numpy()
        tol = max(bar, 4.0 * spread[n])
        err = rel(got, _stack(ref.points, n))
        record(test, 0.0, n, err, tol, spread=spread[n])
        assert err < tol, (n, err, tol)


@pytest.mark.parametrize("b", [4, 40])
def test_loop_fixed_iterations_matches_oracle(nb, b):
    """Four solves with no stopping (tol = 0): the self-energies after three mixings and the Green's
    functions they produced, element by element, plus the residual history."""
    dev = w.folded_chain_device(4, b)
    E, dE, k0, Wl, Wg = _bath(dev, 48)
    scale = 1j * dE / (2 * math.pi)
    ref, spread = _loop_reference(lambda: oscba.scba(dev, E, ETA, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=0.7,
                                                     tol=0.0, max_iter=4))
    res = _gpu_loop(nb, dev, E, Wl, Wg, k0, scale, 0.1, -0.1, mixing=0.7, tol=0.0, max_iter=4)
    assert res["status"] == nb.NEGF_ENOCONV and res["n_iter"] == 4
    assert int(res["info"].abs().sum()) == 0
    _compare_loop(f"scba_fixed_b{b}", res, ref, spread)
    for got, want in zip(res["history"], ref.history):
        assert abs(got - want) <= 1e-8 * want + 1e-12, (res["history"], ref.history)


def test_loop_converges_with_the_oracle(nb):
    """Run to tol = 1e-11: the GPU loop stops at the oracle's iteration (or one apart, when a
    residual sits at the tolerance) at the same fixed point."""
    dev = w.folded_chain_device(4, 24)
    E, dE, k0, Wl, Wg = _bath(dev, 40, n_w=21)
    scale = 1j * dE / (2 * math.pi)
    ref = oscba.scba(dev, E, ETA, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=1.0, tol=1e-11, max_iter=30)
    assert ref.converged
    res = _gpu_loop(nb, dev, E, Wl, Wg, k0, scale, 0.1, -0.1, mixing=1.0, tol=1e-11, max_iter=30)
    assert res["status"] == nb.NEGF_OK, res["history"]
    assert abs(res["n_iter"] - ref.n_iter) <= 1, (res["history"], ref.history)
    for n in ("sig_l", "sig_g"):
        err = rel(res[n].cpu().numpy(), getattr(ref, n))
        record("scba_converged", 0.0, n, err, 1e-9)
        assert err < 1e-9, (n, err)


@pytest.mark.parametrize("b", [4, 40])
def test_loop_anderson_fixed_iterations_matches_oracle(nb, b):
    """Anderson mixing with memory 3 over six solves (five updates, so the history ring wraps once):
    the self-energies and Green's functions element by element against the oracle's loop, and the
    residual history."""
    dev = w.folded_chain_device(4, b)
    E, dE, k0, Wl, Wg = _bath(dev, 48)
    scale = 1j * dE / (2 * math.pi)
    ref, spread = _loop_reference(lambda: oscba.scba(dev, E, ETA, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=0.7,
                                                     tol=0.0, max_iter=6, memory=3))
    res = _gpu_loop(nb, dev, E, Wl, Wg, k0, scale, 0.1, -0.1, mixing=0.7, tol=0.0, max_iter=6, memory=3)
    assert res["status"] == nb.NEGF_ENOCONV and res["n_iter"] == 6
    assert int(res["info"].abs().sum()) == 0
    _compare_loop(f"scba_anderson_fixed_b{b}", res, ref, spread)
    for got, want in zip(res["history"], ref.history):
        assert abs(got - want) <= 1e-8 * want + 1e-12, (res["history"], ref.history)


def test_loop_anderson_converges_where_linear_mixing_diverges(nb):
    """A periodic wire at a coupling where linear mixing (mixing 1) first approaches the fixed point and
    then diverges: the GPU loop with memory 3 converges to the oracle's fixed point (Anderson, memory 3),
    and with linear mixing it does not converge."""
    wire = w.periodic_wire_device(4, 4, 3)
    E = w.energy_grid(-3.0, 3.0, 64)
    dE = float(E[1] - E[0])
    Wl, Wg = w.boson_bath(wire.nb, wire.b, 17, 8, dE, KT, strength=0.2)
    scale = 1j * dE / (2 * math.pi)
    ref = oscba.scba(wire, E, ETA, 0.1, -0.1, KT, Wl, Wg, 8, scale, mixing=1.0, tol=1e-12, max_iter=40, memory=3)
    assert ref.converged
    res = _gpu_loop(nb, wire, E, Wl, Wg, 8, scale, 0.1, -0.1, mixing=1.0, tol=1e-12, max_iter=40, memory=3)
    assert res["status"] == nb.NEGF_OK, res["history"]
    for n in ("sig_l", "sig_g"):
        err = rel(res[n].cpu().numpy(), getattr(ref, n))
        record("scba_anderson_converged", 0.0, n, err, 1e-9)
        assert err < 1e-9, (n, err)
    lin = _gpu_loop(nb, wire, E, Wl, Wg, 8, scale, 0.1, -0.1, mixing=1.0, tol=1e-12, max_iter=40)
    assert lin["status"] != nb.NEGF_OK, lin["history"]


def test_loop_without_bath_is_one_ballistic_solve(nb):
    """W = 0: one solve, zero self-energies, the plain sweeps' result."""
    import torch
    dev = w.folded_chain_device(4, 16)
    E, dE, k0, Wl, Wg = _bath(dev, 20)
    Z = np.zeros_like(Wl)
    res = _gpu_loop(nb, dev, E, Z, Z, k0, 1j * dE / (2 * math.pi), 0.1, -0.1, tol=1e-12, max_iter=5)
    assert res["status"] == nb.NEGF_OK and res["n_iter"] == 1 and res["history"] == [0.0]
    for n in ("sig_r", "sig_l", "sig_g"):
        assert not bool(res[n].abs().max() > 0)
    plain = nb.rgf_lesser_greater([nb.Problem(nb.DeviceOnGPU(dev), E, eta=ETA, mu_l=0.1, mu_r=-0.1, kT=KT)],
                                  greater=True)
    torch.cuda.synchronize()
    for n in ("GR_diag", "GL_diag", "GG_upper"):
        assert rel(res[n][0].cpu().numpy(), plain[n][0].cpu().numpy()) < 1e-13


def test_loop_starts_from_given_self_energies(nb):
    """A start Sigma_0 taken from a converged run is already the fixed point: one solve."""
    dev = w.folded_chain_device(4, 8)
    E, dE, k0, Wl, Wg = _bath(dev, 32)
    scale = 1j * dE / (2 * math.pi)
    ref = oscba.scba(dev, E, ETA, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=1.0, tol=1e-13, max_iter=40)
    res = _gpu_loop(nb, dev, E, Wl, Wg, k0, scale, 0.1, -0.1, sig0=(ref.sig_l, ref.sig_g), tol=1e-11, max_iter=3)
    assert res["status"] == nb.NEGF_OK and res["n_iter"] == 1, res["history"]


# --------------------------------------------------------------- properties at a larger size

def _fermi_residual(E, mu, GL, GG):
    worst = 0.0
    for e in range(len(E)):
        f = oleads.fermi(E[e] - mu, KT)
        scl = np.abs(GL[e]).max() + np.abs(GG[e]).max()
        worst = max(worst, float(np.abs((1 - f) * GL[e] + f * GG[e]).max() / scl))
    return worst


def test_loop_equilibrium_keeps_the_fermi_relation(nb):
    """One Fermi level and a bath at the same temperature: (1 - f) X^< + f X^> = 0 for the
    Green's functions and the self-energies of the last iterate (b = 96, 64 energies)."""
    dev = w.folded_chain_device(6, 96)
    E, dE, k0, Wl, Wg = _bath(dev, 64, n_w=33)
    mu = 0.05
    res = _gpu_loop(nb, dev, E, Wl, Wg, k0, 1j * dE / (2 * math.pi), mu, mu, mixing=0.7, tol=0.0, max_iter=3)
    assert res["n_iter"] == 3
    worst = max(_fermi_residual(E, mu, res["GL_diag"][0].cpu().numpy(), res["GG_diag"][0].cpu().numpy()),
                _fermi_residual(E, mu, res["sig_l"].cpu().numpy(), res["sig_g"].cpu().numpy()))
    record("scba_fermi_relation", mu, "GL/GG", worst, 1e-11)
    assert worst < 1e-11, worst
    assert float(res["sig_l"].abs().max()) > 1e-4


def test_loop_conserves_the_energy_integrated_current(nb):
    """Converged inelastic loop (b = 64): the energy-integrated current is the same at every
    interface and equals the left lead's injection, while the per-energy currents differ."""
    dev = w.folded_chain_device(5, 64)
    E, dE, k0, Wl, Wg = _bath(dev, 64, n_w=25)
    res = _gpu_loop(nb, dev, E, Wl, Wg, k0, 1j * dE / (2 * math.pi), 0.1, -0.1, mixing=1.0, tol=1e-12,
                    max_iter=40)
    assert res["status"] == nb.NEGF_OK, res["history"]
    GLu = res["GL_upper"][0].cpu().numpy()
    GLd = res["GL_diag"][0].cpu().numpy()
    GGd = res["GG_diag"][0].cpu().numpy()
    j = np.array([oobs.currents([E[e] * dev.s_upper(i) - dev.H_upper[i] for i in range(dev.nb - 1)], GLu[e])
                  for e in range(len(E))])
    inj = []
    for e in range(len(E)):
        lead = oleads.lead_self_energy(dev, 0, E[e], ETA)
        sl, sg = oleads.lesser_greater(lead.gamma, oleads.fermi(E[e] - 0.1, KT))
        inj.append(oobs.lead_current(sl, sg, GLd[e][0], GGd[e][0]))
    J, Jin = j.sum(axis=0), float(np.sum(inj))
    err = float(max(np.abs(J - J[0]).max(), abs(J[0] - Jin)) / abs(J[0]))
    record("scba_current_conservation", 0.0, "J", err, 1e-9)
    assert err < 1e-9, (J, Jin)
    assert np.abs(j - j[:, :1]).max() > 1e-4 * np.abs(j).max()


def test_energy_dependent_self_energies_through_a_plan(nb):
    """A plan (two worker streams, graph-replayed chunks of 3 points) reads per-energy
    self-energies like the direct call; its point queue refuses them (a slot takes any task's
    energy), before any work."""
    import torch
    base = w.slab_device(4, 24, 5)
    E = np.linspace(-0.8, 0.9, 7)
    per_e = [w.scattering_self_energies(dataclasses.replace(base), 90 + e, norm=0.02) for e in range(E.size)]
    dev = dataclasses.replace(base, sig_r=np.stack([d.sig_r for d in per_e]), sig_l=np.stack([d.sig_l for d in per_e]),
                              sig_g=np.stack([d.sig_g for d in per_e]))
    prob = nb.Problem(nb.DeviceOnGPU(dev), E, eta=ETA, mu_l=0.1, mu_r=-0.1, kT=KT, sc_stride=4 * 24 * 24)
    direct = nb.rgf_lesser_greater([prob], greater=True)
    plan = nb.Plan([prob], opts=nb.make_options(batch=3), n_streams=2)
    outs = plan.outputs(greater=True)
    info = torch.zeros(E.size, dtype=torch.int32, device="cuda")
    plan.execute(outs, info, use_graph=True)
    torch.cuda.synchronize()
    assert int(info.abs().sum()) == 0
    for n in ("GR_diag", "GR_upper", "GL_diag", "GL_upper", "GG_diag"):
        a, b = outs[n].cpu().numpy(), direct["flat"][n].cpu().numpy()
        assert rel(a, b) < 1e-13, n
    with pytest.raises(nb.NegfError):
        plan.run_queue([torch.tensor([0.1, 0.2], dtype=torch.float64, device="cuda")], outs, info)
    plan.close()


# --------------------------------------------------------------- the loop as single captured steps

def _step_loop(nb, dev, E, Wl, Wg, k0, scale, mixing, tol, max_steps, memory=0):
    import torch
    prob = nb.Problem(nb.DeviceOnGPU(dev), E, eta=ETA, mu_l=0.1, mu_r=-0.1, kT=KT)
    return nb.ScbaLoop(prob, torch.from_numpy(Wl).cuda(), torch.from_numpy(Wg).cuda(), k0, scale, mixing=mixing,
                       tol=tol, max_steps=max_steps, memory=memory)


@pytest.mark.parametrize("tol,steps,memory", [(0.0, 4, 0), (1e-11, 16, 0), (0.0, 7, 2), (1e-11, 16, 3)])
def test_loop_steps_equal_the_driver_and_replay_from_a_graph(nb, tol, steps, memory):
    """negf_scba_step run `steps` times (the last without mixing) ends on exactly what negf_scba ends on:
    with tol = 0 after the same four solves; with tol = 1e-11 the steps after convergence leave the
    self-energies alone and recompute the same Green's functions.  The same steps captured once in a
    graph and replayed (self-energies cleared between replays) give the same bits again.  With an
    Anderson memory the history in the workspace is rebuilt by every run from its first step, so the
    replays match as well."""
    import torch
    dev = w.folded_chain_device(4, 24)
    E, dE, k0, Wl, Wg = _bath(dev, 40, n_w=21)
    scale = 1j * dE / (2 * math.pi)
    ref = _gpu_loop(nb, dev, E, Wl, Wg, k0, scale, 0.1, -0.1, mixing=1.0, tol=tol, max_iter=steps, memory=memory)
    loop = _step_loop(nb, dev, E, Wl, Wg, k0, scale, 1.0, tol, steps, memory=memory)
    loop.run(steps)
    torch.cuda.synchronize()
    names = ("sig_r", "sig_l", "sig_g")
    outs = ("GR_diag", "GR_upper", "GL_diag", "GL_upper", "GG_diag", "GG_upper")
    st = loop.state.cpu().tolist()
    assert st[0] == ref["n_iter"], (st, ref["n_iter"])
    assert st[1] == (1 if ref["status"] == nb.NEGF_OK else 0), (st, ref["status"])
    assert loop.history[:ref["n_iter"]].cpu().tolist() == ref["history"]
    for n in names:
        assert torch.equal(loop.sig[n], ref[n]), n
    for n in outs:
        assert torch.equal(loop.out[n], ref["flat"][n]), n
    eager = {n: loop.sig[n].clone() for n in names}
    eager.update({n: loop.out[n].clone() for n in outs})
    # capture the whole loop once
    for n in names:
        loop.sig[n].zero_()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        loop.run(steps)
    torch.cuda.current_stream().wait_stream(side)
    for n in names:
        loop.sig[n].zero_()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        loop.run(steps)
    for rep in range(2):
        for n in names:
            loop.sig[n].zero_()
        for n in outs:
            loop.out[n].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for n in names:
            assert torch.equal(loop.sig[n], eager[n]), (rep, n)
        for n in outs:
            assert torch.equal(loop.out[n], eager[n]), (rep, n)
        assert loop.state.cpu().tolist() == st, rep
    del g


def test_loop_in_the_refined_form_and_in_chunks(nb):
    """The loop's solves in the refined single-product form stay within its 1e-6 bar of the oracle loop
    (plain arithmetic) after three iterations; with the solves split into chunks of 5 energies (so that
    chunks start inside the self-energy arrays) the plain loop is unchanged to 1e-13."""
    import torch
    dev = w.slab_device(4, 32, 8)
    E, dE, k0, Wl, Wg = _bath(dev, 24, lo=-0.6, hi=0.6, n_w=9, strength=0.3)
    scale = 1j * dE / (2 * math.pi)
    ref = oscba.scba(dev, E, ETA, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=0.7, tol=0.0, max_iter=3)
    plain = _gpu_loop(nb, dev, E, Wl, Wg, k0, scale, 0.1, -0.1, mixing=0.7, tol=0.0, max_iter=3)
    refined = _gpu_loop(nb, dev, E, Wl, Wg, k0, scale, 0.1, -0.1, mixing=0.7, tol=0.0, max_iter=3, prec=nb.FP32_REFINE)
    chunked = _gpu_loop(nb, dev, E, Wl, Wg, k0, scale, 0.1, -0.1, mixing=0.7, tol=0.0, max_iter=3,
                        opts=nb.make_options(batch=5))
    for n in ("sig_l", "sig_g"):
        err = rel(refined[n].cpu().numpy(), getattr(ref, n))
        record("scba_refined_form", 0.0, n, err, 1e-6)
        assert err < 1e-6, (n, err)
        assert rel(chunked[n].cpu().numpy(), plain[n].cpu().numpy()) < 1e-13, n
    for n in ("GR_diag", "GL_diag", "GG_diag"):
        err = rel(refined[n][0].cpu().numpy(), _stack(ref.points, n))
        record("scba_refined_form", 0.0, n, err, 1e-6)
        assert err < 1e-6, (n, err)
        assert rel(chunked[n][0].cpu().numpy(), plain[n][0].cpu().numpy()) < 1e-13, n


def _k_devices(b):
    base = w.folded_chain_device(4, b)
    T = 0.2 * np.eye(b, k=1)
    devs = []
    for kk in (0.0, 1.3):
        ph = complex(math.cos(kk), math.sin(kk))
        devs.append(w.BTDevice(np.stack([h + ph * T + np.conj(ph) * T.T for h in base.H_diag]), base.H_upper))
    return base, devs


@pytest.mark.parametrize("b", [4, 24])
def test_loop_over_k_points_matches_oracle(nb, b):
    """Two transverse momenta sharing k-independent self-energies built from their average G^<>: the
    self-energies and every k-point's Green's functions after three solves against the oracle loop;
    the same device given twice reproduces the single-device loop bit for bit."""
    import torch
    base, devs = _k_devices(b)
    E, dE, k0, Wl, Wg = _bath(base, 32, n_w=9)
    scale = 1j * dE / (2 * math.pi)
    ref = oscba.scba(devs, E, ETA, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=0.7, tol=0.0, max_iter=3)
    probs = [nb.Problem(nb.DeviceOnGPU(d), E, eta=ETA, mu_l=0.1, mu_r=-0.1, kT=KT) for d in devs]
    gWl, gWg = torch.from_numpy(Wl).cuda(), torch.from_numpy(Wg).cuda()
    res = nb.scba(probs, gWl, gWg, k0, scale, mixing=0.7, tol=0.0, max_iter=3)
    torch.cuda.synchronize()
    assert res["n_iter"] == 3 and int(res["info"].abs().sum()) == 0
    for n in ("sig_l", "sig_g", "sig_r"):
        err = rel(res[n].cpu().numpy(), getattr(ref, n))
        record(f"scba_k_points_b{b}", 0.0, n, err, 1e-10)
        assert err < 1e-10, (n, err)
    for q in range(len(devs)):
        for n in ("GR_diag", "GL_diag", "GL_upper", "GG_diag"):
            err = rel(res[n][q].cpu().numpy(), _stack(ref.points[q], n))
            record(f"scba_k_points_b{b}", 0.0, n, err, 1e-10)
            assert err < 1e-10, (q, n, err)
    one = nb.scba(probs[0], gWl, gWg, k0, scale, mixing=0.7, tol=0.0, max_iter=3)
    twice = nb.scba([probs[0], probs[0]], gWl, gWg, k0, scale, mixing=0.7, tol=0.0, max_iter=3)
    torch.cuda.synchronize()
    for n in ("sig_l", "sig_g", "sig_r"):
        assert torch.equal(one[n], twice[n]), n


def test_loop_anderson_over_k_points_and_in_the_refined_form(nb):
    """Anderson mixing (memory 2) over two k-points: five solves against the oracle's Anderson loop
    (plain 1e-10); the same loop with its solves in the refined single-product form within that form's
    1e-6 bar."""
    import torch
    base, devs = _k_devices(4)
    E, dE, k0, Wl, Wg = _bath(base, 32, n_w=9)
    scale = 1j * dE / (2 * math.pi)
    ref = oscba.scba(devs, E, ETA, 0.1, -0.1, KT, Wl, Wg, k0, scale, mixing=0.7, tol=0.0, max_iter=5, memory=2)
    probs = [nb.Problem(nb.DeviceOnGPU(d), E, eta=ETA, mu_l=0.1, mu_r=-0.1, kT=KT) for d in devs]
    gWl, gWg = torch.from_numpy(Wl).cuda(), torch.from_numpy(Wg).cuda()
    print(f"  negf_scba over {len(devs)} k-points, memory 2, plain and refined", flush=True)
    res = nb.scba(probs, gWl, gWg, k0, scale, mixing=0.7, tol=0.0, max_iter=5, memory=2)
    fine = nb.scba(probs, gWl, gWg, k0, scale, mixing=0.7, tol=0.0, max_iter=5, memory=2, prec=nb.FP32_REFINE)
    torch.cuda.synchronize()
    assert res["n_iter"] == 5 and int(res["info"].abs().sum()) == 0
    for got, bar, name in ((res, 1e-10, "scba_anderson_k_points"), (fine, 1e-6, "scba_anderson_k_points_refine")):
        for n in ("sig_l", "sig_g", "sig_r"):
            err = rel(got[n].cpu().numpy(), getattr(ref, n))
            record(name, 0.0, n, err, bar)
            assert err < bar, (name, n, err)
        for q in range(len(devs)):
            for n in ("GR_diag", "GL_diag", "GG_diag"):
                err = rel(got[n][q].cpu().numpy(), _stack(ref.points[q], n))
                record(name, 0.0, n, err, bar)
                assert err < bar, (name, q, n, err)


def test_loop_over_k_points_conserves_the_summed_current(nb):
    """Converged over two k-points (b = 24): the energy-integrated current summed over the k-points is the
    same at every interface (negf_observables on the loop's outputs)."""
    import torch
    base, devs = _k_devices(24)
    E, dE, k0, Wl, Wg = _bath(base, 40, n_w=13)
    probs = [nb.Problem(nb.DeviceOnGPU(d), E, eta=ETA, mu_l=0.1, mu_r=-0.1, kT=KT) for d in devs]
    res = nb.scba(probs, torch.from_numpy(Wl).cuda(), torch.from_numpy(Wg).cuda(), k0, 1j * dE / (2 * math.pi),
                  mixing=1.0, tol=1e-12, max_iter=40)
    assert res["status"] == nb.NEGF_OK, res["history"]
    cur = nb.observables(probs, res["flat"], dos=False)["current"]
    J = sum(c.cpu().numpy().sum(axis=0) for c in cur)
    err = float(np.abs(J - J[0]).max() / abs(J[0]))
    record("scba_k_points_current", 0.0, "J", err, 1e-9)
    assert err < 1e-9, J


def test_loop_reports_a_non_finite_residual(nb):
    """A NaN in the bath makes the first residual non-finite: negf_scba returns ENONFINITE after that
    solve, and the self-energies are left as they were (the mixing pass reads the state)."""
    import torch
    dev = w.folded_chain_device(4, 8)
    E, dE, k0, Wl, Wg = _bath(dev, 20)
    Wl = Wl.copy()
    Wl[k0, 1, 2, 3] = np.nan
    res = _gpu_loop(nb, dev, E, Wl, Wg, k0, 1j * dE / (2 * math.pi), 0.1, -0.1, tol=1e-12, max_iter=5)
    assert res["status"] == nb.NEGF_ENONFINITE and res["n_iter"] == 1, (res["status"], res["history"])
    assert not math.isfinite(res["history"][0])
    for n in ("sig_r", "sig_l", "sig_g"):
        assert not bool(res[n].abs().max() > 0), n          # still the zero start
