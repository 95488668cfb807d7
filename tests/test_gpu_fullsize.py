"""GPU parity at the full benchmark size: Nb = 60 blocks of b = 512.

The headline path is what ``bench.py`` times: one call of
negf_rgf_lesser_greater over one chunk of 128 energy points on one stream,
with the benchmark's options (decimation step count, tile, panel width,
three-product complex products).  The plan path (two worker streams, 64
points) is checked beside it.

The oracle takes seconds per point at this size, so a sample of points is
compared element by element; every point of a batch is checked for properties
that hold at any size: G^<_ii is anti-Hermitian and the local density of
states -Im Tr G^R_ii / pi is non-negative.

Two broadenings of the leads:
  eta = 1e-2  The oracle is stable to the plain bar at the sampled points (its
              outputs move by <= 1.3e-11 when its inversions are refined), so
              the headline path is held to the fixed 1e-10.
  eta = 1e-8  The benchmark's own setting.  At this size no energy of the grid
              has both lead decimations stable to 2.5e-11 under refined
              inversions (a scan of 16 grid energies: 1e-10 .. 3e-7), so each
              sampled point is held to max(1e-10, 4 x the oracle's spread),
              printed and recorded.  The decimation of these random leads is
              ill-conditioned at a few energies (the oracle itself ends with a
              Dyson residual of 1e-9 .. 1e-8 there, or diverges): the GPU flags
              them ENOCONV, and the test requires every flagged point to be
              one where the oracle's own decimation is not clean and every
              sampled clean point to be unflagged.
"""
import dataclasses
import os
import time

import numpy as np
import pytest

import workloads as w
from helpers import kappa_proxy, oracle_spread, plain_reference, record, well_posed, SPREAD_FACTOR
from oracle import leads as oleads
from oracle import econv as oecv
from oracle import rgf as orgf

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

NB, B = 60, 512
P_HEADLINE, P_PLAN, PLAN_STREAMS = 128, 64, 2
ETA, MU_L, MU_R, KT = 1e-8, 0.1, -0.1, 0.025
ETA_STABLE = 1e-2
# points of the first benchmark batch sampled at eta = 1e-2 (energies -1.031, 0.095, 0.471, 1.221)
STABLE_K = (20, 68, 84, 116)
CLEAN = 1e-10
PLAIN_TOL = 1e-10
NAMES = ["GR_diag", "GR_upper", "GR_lower", "GL_diag", "GL_upper"]
_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _progress(msg):
    """Oracle evaluations at this size take a while: each one leaves a line."""
    d = os.path.join(_ROOT, "gpurun_out", "parity")
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "fullsize_progress.log"), "a") as fh:
        fh.write(f"{time.strftime('%H:%M:%S')} {msg}\n")
    print(msg, flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import bench
    from paper_2602_03438_amd import autotune
    from paper_2602_03438_amd import binding as nb
    nb.lib()
    dev = w.slab_device(NB, B, 2)
    gdev = nb.DeviceOnGPU(dev)
    energies = bench.energy_batches(P_HEADLINE)[0]
    yield nb, bench, autotune, dev, gdev, energies
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _headline_opts(nb, bench, autotune, cmul=3):
    t = autotune.lookup(B, cmul)
    return nb.make_options(inv_nb=t["inv_nb"], cmul=cmul, gemm_tile=t["gemm_tile"], gemm_tile_f32=t["gemm_tile_f32"],
                           sr_max_iter=40)


def _run(nb, bench, prob, prec, opts, streams, points):
    """One step of the benchmark's runner; returns (outputs, info)."""
    import torch
    outputs = nb._rgf_outputs([prob], True, False, True)
    run, plan = bench.make_runner(nb, [prob], prec, outputs, None, opts, streams, points)
    info = run()
    torch.cuda.synchronize()
    if plan:
        plan.close()
    return outputs, info.cpu().numpy()


def _free():
    import gc
    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _point(nb, outputs, prob, k, name):
    return nb._views(outputs, [prob])[name][0][k].cpu().numpy()


def _clean(dev, E):
    """Both lead decimations of the oracle converge to a residual <= CLEAN."""
    for side in (0, 1):
        r = oleads.lead_self_energy(dev, side, E, ETA)
        if not (r.converged and r.residual <= CLEAN):
            return False
    return True


def _properties(nb, outputs, prob, info):
    import torch
    v = nb._views(outputs, [prob])
    for k in range(prob.n_e):
        if info[k] != 0:
            continue
        gl = v["GL_diag"][0][k]
        skew = torch.linalg.vector_norm(gl + gl.transpose(-1, -2).conj()) / torch.linalg.vector_norm(gl)
        # exact in exact arithmetic; rounding amplified by the ill-conditioned
        # sweeps of this workload reaches ~3e-10, a wrong term gives O(1)
        assert skew.item() < 1e-8, (k, skew.item())
        ldos = -torch.diagonal(v["GR_diag"][0][k], dim1=-2, dim2=-1).imag.sum(-1)
        scale = torch.diagonal(v["GR_diag"][0][k], dim1=-2, dim2=-1).abs().sum(-1)
        assert torch.all(ldos >= -1e-10 * scale).item(), k


def _compare(nb, outputs, prob, energies, refs, test, names=NAMES):
    for k, (ref, bars, spread, kappa) in refs.items():
        for name in names:
            g = _point(nb, outputs, prob, k, name)
            r = getattr(ref, name)
            err = float(np.linalg.norm(g - r) / np.linalg.norm(r))
            bar = bars[name] if isinstance(bars, dict) else bars
            record(test, energies[k], name, err, bar, spread.get(name), kappa, point=int(k))
            _progress(f"{test} point {k} (E = {energies[k]:+.6f}) {name}: error {err:.3e}, bar {bar:.1e}, "
                      f"oracle spread {spread.get(name, float('nan')):.1e}")
            assert err <= bar, (test, k, name, err, bar)


# ------------------------------------------------------------------ eta = 1e-2: the plain bar

@pytest.fixture(scope="module")
def stable_refs(setup):
    nb, bench, autotune, dev, gdev, energies = setup
    out = {}
    for k in STABLE_K:
        _progress(f"oracle at eta = {ETA_STABLE}, point {k} (E = {energies[k]:+.6f}) ...")
        ref, spread = plain_reference(lambda: orgf.solve_point(dev, energies[k], ETA_STABLE, MU_L, MU_R, KT), NAMES,
                                      PLAIN_TOL)
        out[k] = (ref, PLAIN_TOL, spread, kappa_proxy(dev, ref))
    return out


def test_fullsize_headline_path_plain_bar(setup, stable_refs):
    """The benchmark's call (one chunk of 128 points, one stream) at eta = 1e-2,
    where the oracle referees the plain 1e-10 bar."""
    nb, bench, autotune, dev, gdev, energies = setup
    prob = nb.Problem(gdev, energies, eta=ETA_STABLE, mu_l=MU_L, mu_r=MU_R, kT=KT)
    outputs, info = _run(nb, bench, prob, nb.PLAIN_FP64, _headline_opts(nb, bench, autotune), 1, P_HEADLINE)
    assert np.all(info == 0), np.nonzero(info)[0]
    _compare(nb, outputs, prob, energies, stable_refs, "fullsize_headline_eta1e-2")
    _properties(nb, outputs, prob, info)
    # every point: the spectral current (negf_observables) is the same at all 59 interfaces
    cur = nb.observables([prob], outputs, dos=False)["current"][0].cpu().numpy()
    scale = float(np.abs(cur).max())
    spread = float(np.abs(cur - cur[:, :1]).max() / scale)
    record("fullsize_current_conservation_eta1e-2", 0.0, "current", spread, 1e-8, points=int(cur.shape[0]))
    _progress(f"current conservation over {cur.shape[0]} points x {cur.shape[1]} interfaces: {spread:.2e} of the "
              f"largest current")
    assert spread < 1e-8, spread
    del outputs
    _free()


def test_fullsize_headline_refined_form_plain_eta(setup, stable_refs):
    """The refined single-product form on the same call, every output kind at 1e-6."""
    nb, bench, autotune, dev, gdev, energies = setup
    prob = nb.Problem(gdev, energies, eta=ETA_STABLE, mu_l=MU_L, mu_r=MU_R, kT=KT)
    outputs, info = _run(nb, bench, prob, nb.FP32_REFINE, _headline_opts(nb, bench, autotune), 1, P_HEADLINE)
    assert np.all(info == 0)
    refs = {k: (ref, 1e-6, spread, kappa) for k, (ref, _, spread, kappa) in stable_refs.items()}
    _compare(nb, outputs, prob, energies, refs, "fullsize_headline_fp32_refine_eta1e-2")
    del outputs
    _free()


# ------------------------------------------------------------------ eta = 1e-8: the benchmark setting

def _sample(dev, energies, n=4):
    """n clean, well-posed points spread over the batch."""
    picks = []
    step = len(energies) // n
    for s in range(n):
        for k in range(s * step + step // 3, (s + 1) * step):
            if _clean(dev, energies[k]) and well_posed(dev, energies[k:k + 1]).size:
                picks.append(k)
                break
    assert len(picks) == n
    return picks


@pytest.fixture(scope="module")
def refs(setup):
    """Oracle results and per-point bars at sampled clean points at eta = 1e-8."""
    nb, bench, autotune, dev, gdev, energies = setup
    out = {}
    for k in _sample(dev, energies):
        _progress(f"oracle at eta = {ETA}, point {k} (E = {energies[k]:+.6f}) ...")
        ref, spread = oracle_spread(lambda: orgf.solve_point(dev, energies[k], ETA, MU_L, MU_R, KT), NAMES)
        bars = {n: max(PLAIN_TOL, SPREAD_FACTOR * spread[n]) for n in NAMES}
        out[k] = (ref, bars, spread, kappa_proxy(dev, ref))
    return out


def _flags_justified(dev, energies, info, refs, points):
    for k in refs:
        assert info[k] == 0, (k, energies[k], info[k])
    flagged = np.nonzero(info[:points])[0]
    assert flagged.size <= points // 8, flagged
    for k in flagged:
        assert info[k] == 2, (k, info[k])          # ENOCONV, not a singular or non-finite sweep
        assert not _clean(dev, energies[k]), (k, energies[k])


def test_fullsize_headline_path_conditioned(setup, refs):
    """The benchmark's call at its own eta = 1e-8."""
    nb, bench, autotune, dev, gdev, energies = setup
    prob = nb.Problem(gdev, energies, eta=ETA, mu_l=MU_L, mu_r=MU_R, kT=KT)
    outputs, info = _run(nb, bench, prob, nb.PLAIN_FP64, _headline_opts(nb, bench, autotune), 1, P_HEADLINE)
    _progress(f"flagged points: {np.nonzero(info)[0].tolist()}")
    _flags_justified(dev, energies, info, refs, P_HEADLINE)
    _compare(nb, outputs, prob, energies, refs, "fullsize_headline_eta1e-8_conditioned")
    _properties(nb, outputs, prob, info)
    del outputs
    _free()


def test_fullsize_headline_refined_form_conditioned(setup, refs):
    nb, bench, autotune, dev, gdev, energies = setup
    prob = nb.Problem(gdev, energies, eta=ETA, mu_l=MU_L, mu_r=MU_R, kT=KT)
    outputs, info = _run(nb, bench, prob, nb.FP32_REFINE, _headline_opts(nb, bench, autotune), 1, P_HEADLINE)
    for k in refs:
        assert info[k] == 0, (k, info[k])
    rr = {k: (ref, 1e-6, spread, kappa) for k, (ref, _, spread, kappa) in refs.items()}
    _compare(nb, outputs, prob, energies, rr, "fullsize_headline_fp32_refine_eta1e-8")
    del outputs
    _free()


@pytest.mark.parametrize("cmul", [4, 3])
def test_fullsize_plan_path_conditioned(setup, refs, cmul):
    """Two worker streams over the first 64 points (the plan path)."""
    nb, bench, autotune, dev, gdev, energies = setup
    e64 = energies[:P_PLAN]
    prob = nb.Problem(gdev, e64, eta=ETA, mu_l=MU_L, mu_r=MU_R, kT=KT)
    opts = nb.make_options(inv_nb=16, cmul=cmul)
    outputs, info = _run(nb, bench, prob, nb.PLAIN_FP64, opts, PLAN_STREAMS, P_PLAN)
    sub = {k: v for k, v in refs.items() if k < P_PLAN}
    assert sub, "no sampled point in the first half"
    _flags_justified(dev, e64, info, sub, P_PLAN)
    _compare(nb, outputs, prob, e64, sub, f"fullsize_plan_eta1e-8_conditioned_cmul{cmul}")
    _properties(nb, outputs, prob, info)
    del outputs
    _free()


@pytest.fixture(scope="module")
def scattering_refs(setup):
    """The same device with the scattering self-energies of the interacting
    workload (norm 0.01), oracle at two sampled energies at eta = 1e-2."""
    nb, bench, autotune, dev, gdev, energies = setup
    sdev = w.scattering_self_energies(w.slab_device(NB, B, 2), 3)
    out = {}
    for k in STABLE_K[:2]:
        _progress(f"oracle (scattering device) at eta = {ETA_STABLE}, point {k} (E = {energies[k]:+.6f}) ...")
        ref, spread = plain_reference(lambda: orgf.solve_point(sdev, energies[k], ETA_STABLE, MU_L, MU_R, KT),
                                      NAMES, PLAIN_TOL)
        out[k] = (ref, PLAIN_TOL, spread, kappa_proxy(sdev, ref))
    return sdev, out


@pytest.mark.parametrize("parts", [8, 4])
def test_fullsize_serinv_plain_bar(setup, scattering_refs, parts):
    """The partitioned inversion at the full size (eight or four partitions of
    the 60 blocks, two energies in one call) against the oracle at eta = 1e-2,
    on the device with scattering self-energies: the partitions' interiors are
    then broadened like every other block.  (Without any broadening inside the
    device, an isolated interior at a real energy is nearly singular and the
    partitioned elimination loses up to ~1e-7 at this size, the oracle's own
    partitioned prototype included.)"""
    nb, bench, autotune, dev, gdev, energies = setup
    sdev, refs = scattering_refs
    ks = sorted(refs)
    prob = nb.Problem(nb.DeviceOnGPU(sdev), energies[ks], eta=ETA_STABLE, mu_l=MU_L, mu_r=MU_R, kT=KT)
    out = nb.serinv_lesser_greater(prob, parts, opts=_headline_opts(nb, bench, autotune))
    info = out["info"].cpu().numpy()
    assert np.all(info == 0), info
    for i, k in enumerate(ks):
        ref, bar, spread, kappa = refs[k]
        for name in NAMES:
            g = out[name][0][i].cpu().numpy()
            r = getattr(ref, name)
            err = float(np.linalg.norm(g - r) / np.linalg.norm(r))
            record(f"fullsize_serinv_P{parts}_scattering_eta1e-2", energies[k], name, err, bar, spread.get(name),
                   kappa, partitions=parts)
            _progress(f"serinv P={parts} point {k} {name}: error {err:.3e}, bar {bar:.1e}")
            assert err <= bar, (parts, k, name, err)
    del out
    _free()


# ------------------------------------------------------------------ the self-consistent loop at full size

def test_fullsize_self_consistent_loop_plain_bar(setup):
    """negf_scba at the benchmark's shape and options (Nb = 60, b = 512, three-product complex
    products), eta = 1e-2: two iterations from zero self-energies over 8 energies, a bath of 3
    frequencies.  After them the self-energies are m F_0, with F_0 the Eq. (3) convolution of the
    ballistic G^<> (the oracle solves the three energies the sampled energy's window reaches and
    convolves them), and the Green's functions at the sampled energy are the oracle's solve with
    the oracle's self-energies there.  The oracle is stable to the plain bar at these points
    (asserted through its spread)."""
    import torch
    nb, bench, autotune, dev, gdev, _ = setup
    n_e, n_w, k0, es, m = 8, 3, 1, 4, 0.5
    E = 0.095 + (np.arange(n_e) - 4) * 0.03
    dE = float(E[1] - E[0])
    Wl, Wg = w.boson_bath(NB, B, n_w, k0, dE, KT, strength=0.05)
    scale = 1j * dE / (2 * np.pi)
    prob = nb.Problem(gdev, E, eta=ETA_STABLE, mu_l=MU_L, mu_r=MU_R, kT=KT)
    _progress("negf_scba at full size: 8 energies, bath of 3 frequencies, 2 iterations ...")
    res = nb.scba(prob, torch.from_numpy(Wl).cuda(), torch.from_numpy(Wg).cuda(), k0, scale, mixing=m, tol=0.0,
                  max_iter=2, opts=_headline_opts(nb, bench, autotune))
    torch.cuda.synchronize()
    assert res["n_iter"] == 2 and res["status"] == nb.NEGF_ENOCONV
    assert int(res["info"].abs().sum()) == 0
    # the oracle's ballistic G^<> on the window es - k0 .. es + k0 and its convolution at es
    win = range(es - k0, es + n_w - k0)
    Gl, Gg, spread0 = [], [], 0.0
    for e in win:
        _progress(f"oracle (ballistic) at E = {E[e]:+.4f} ...")
        ref, sp = plain_reference(lambda: orgf.solve_point(dev, E[e], ETA_STABLE, MU_L, MU_R, KT, greater=True),
                                  ["GL_diag", "GG_diag"], PLAIN_TOL)
        Gl.append(ref.GL_diag)
        Gg.append(ref.GG_diag)
        spread0 = max(spread0, *sp.values())
        del ref
    Gl, Gg = np.stack(Gl), np.stack(Gg)
    n_el = NB * B * B
    j = es - win.start
    Sl = m * oecv.energy_convolution(Gl.reshape(n_w, n_el), Wl.reshape(n_w, n_el), k0, scale)[j].reshape(NB, B, B)
    Sg = m * oecv.energy_convolution(Gg.reshape(n_w, n_el), Wg.reshape(n_w, n_el), k0, scale)[j].reshape(NB, B, B)
    del Gl, Gg
    for name, want in (("sig_l", Sl), ("sig_g", Sg), ("sig_r", 0.5 * (Sg - Sl))):
        got = res[name][es].cpu().numpy()
        err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        record("fullsize_scba_eta1e-2", E[es], name, err, PLAIN_TOL, spread0)
        _progress(f"scba self-energy {name} at E = {E[es]:+.4f}: error {err:.3e}, bar {PLAIN_TOL:.1e}")
        assert err <= PLAIN_TOL, (name, err)
    # the Green's functions at es: the oracle's solve with the oracle's self-energies
    sdev = dataclasses.replace(dev, sig_r=0.5 * (Sg - Sl), sig_l=Sl, sig_g=Sg)
    names = NAMES + ["GG_diag"]
    _progress(f"oracle (with the loop's self-energies) at E = {E[es]:+.4f} ...")
    ref, sp = plain_reference(lambda: orgf.solve_point(sdev, E[es], ETA_STABLE, MU_L, MU_R, KT, greater=True), names,
                              PLAIN_TOL)
    for name in names:
        got = res[name][0][es].cpu().numpy()
        want = getattr(ref, name)
        err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
        record("fullsize_scba_eta1e-2", E[es], name, err, PLAIN_TOL, sp.get(name))
        _progress(f"scba {name} at E = {E[es]:+.4f}: error {err:.3e}, bar {PLAIN_TOL:.1e}")
        assert err <= PLAIN_TOL, (name, err)
    del res
    _free()
