"""The library's host orchestration, run on the CPU with the test double of its
kernels (tests/hostsim), against the oracle.

This checks the sequencing of the batched launches (operand order, conjugate
transposes, strides, chunking, workspace carving, masks and info codes)
without a GPU; the HIP kernels themselves are checked by the gpu tests.
"""
import ctypes as C
import dataclasses
import os

import numpy as np
import pytest

import workloads as w
from oracle import leads as oleads
from oracle import rgf as orgf
from helpers import point_tolerance, well_posed

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def sim():
    from paper_2602_03438_amd import binding as nb
    import importlib.util
    spec = importlib.util.spec_from_file_location("hostsim_build", os.path.join(HERE, "hostsim", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    path = mod.build(sanitize=os.environ.get("NEGF_HOSTSIM_SANITIZED") == "1")
    L = C.CDLL(path)
    P = C.POINTER
    vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    L.negf_workspace_bytes.argtypes = [i32, P(nb.negf_problem), i32, i32, P(nb.negf_options)]
    L.negf_workspace_bytes.restype = sz
    L.negf_obc_surface.argtypes = [P(nb.negf_problem), i32, i32, P(nb.negf_options), vp, vp, vp, vp, vp, vp, vp, sz,
                                   vp]
    L.negf_rgf_retarded.argtypes = [P(nb.negf_problem), i32, i32, P(nb.negf_options), vp, vp, vp, vp, vp, sz, vp]
    L.negf_rgf_lesser_greater.argtypes = [P(nb.negf_problem), i32, i32, P(nb.negf_options), vp, vp, vp, vp, vp, vp,
                                          vp, vp, vp, sz, vp]
    L.negf_transmission.argtypes = [P(nb.negf_problem), i32, P(nb.negf_options), vp, vp, vp, sz, vp]
    L.negf_plan_create.argtypes = [P(nb.negf_problem), i32, i32, P(nb.negf_options), vp, i32, i32, P(vp)]
    L.negf_plan_workspace_bytes.argtypes = [vp]
    L.negf_plan_workspace_bytes.restype = sz
    L.negf_plan_chunks.argtypes = [vp, vp, vp, vp]
    L.negf_plan_execute.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.negf_plan_destroy.argtypes = [vp]
    return L, nb


class HostProblem:
    def __init__(self, nb, dev, energies, eta=1e-8, mu_l=0.1, mu_r=-0.1, kT=0.025, sc_stride=0):
        self.keep = [np.ascontiguousarray(x) if x is not None else None
                     for x in (dev.H_diag, dev.H_upper, dev.S_diag, dev.S_upper, dev.sig_r, dev.sig_l, dev.sig_g)]
        self.E = np.ascontiguousarray(energies, dtype=np.float64)
        ptr = lambda a: a.ctypes.data if a is not None else None
        d = nb.negf_device(dev.nb, dev.b, *[ptr(a) for a in self.keep])
        self.s = nb.negf_problem(d, self.E.size, self.E.ctypes.data, eta, mu_l, mu_r, kT, sc_stride)
        self.nb, self.b, self.n = dev.nb, dev.b, self.E.size


def _run_rgf(L, nb, probs, prec=0, greater=True, opts=None):
    arr = (nb.negf_problem * len(probs))(*[p.s for p in probs])
    o = C.byref(opts) if opts is not None else None
    ws = np.zeros(L.negf_workspace_bytes(nb.OP_LESSER_GREATER, arr, len(probs), prec, o) + 256, dtype=np.uint8)
    nd = sum(p.n * p.nb * p.b * p.b for p in probs)
    nu = sum(p.n * (p.nb - 1) * p.b * p.b for p in probs)
    out = {k: np.zeros(nd if k.endswith("d") else nu, dtype=np.complex128)
           for k in ("GRd", "GRu", "GRl", "GLd", "GLu", "GGd", "GGu")}
    info = np.zeros(sum(p.n for p in probs), dtype=np.int32)
    g = lambda k: out[k].ctypes.data if (greater or not k.startswith("GG")) else None
    code = L.negf_rgf_lesser_greater(arr, len(probs), prec, o, g("GRd"), g("GRu"), g("GRl"), g("GLd"), g("GLu"),
                                     g("GGd"), g("GGu"), info.ctypes.data, ws.ctypes.data, ws.size, None)
    assert code == 0
    return out, info


def _unpack(flat, probs, diag):
    res, off = [], 0
    for p in probs:
        k = p.nb if diag else p.nb - 1
        n = p.n * k * p.b * p.b
        res.append(flat[off:off + n].reshape(p.n, k, p.b, p.b))
        off += n
    return res


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("scatter", [False, True])
def test_hostsim_lesser_greater_matches_oracle(sim, scatter):
    L, nb = sim
    dev = w.random_device(4, 5, 3, overlap=0.05)
    if scatter:
        w.scattering_self_energies(dev, 4, norm=0.05)
    E = well_posed(dev, np.linspace(-1.2, 1.2, 9))[:3]
    assert E.size == 3
    p = HostProblem(nb, dev, E)
    out, info = _run_rgf(L, nb, [p])
    assert np.all(info == 0)
    for name, ref_name, diag in (("GRd", "GR_diag", 1), ("GRu", "GR_upper", 0), ("GRl", "GR_lower", 0),
                                 ("GLd", "GL_diag", 1), ("GLu", "GL_upper", 0), ("GGd", "GG_diag", 1),
                                 ("GGu", "GG_upper", 0)):
        got = _unpack(out[name], [p], diag)[0]
        for k, e in enumerate(E):
            ref = getattr(orgf.solve_point(dev, e, 1e-8, 0.1, -0.1, 0.025, greater=True), ref_name)
            assert rel(got[k], ref) < 1e-11, (name, k)


def test_hostsim_energy_dependent_self_energies(sim):
    """sc_stride: every energy reads its own scattering self-energies, also when its problem's
    energies are split over chunks (batch 2) that they share with another problem."""
    L, nb = sim
    base = w.random_device(4, 5, 3, overlap=0.05)
    E = well_posed(base, np.linspace(-1.2, 1.2, 13))[:5]
    assert E.size == 5
    per_e = [w.scattering_self_energies(dataclasses.replace(base), 20 + e, norm=0.05) for e in range(E.size)]
    dev = dataclasses.replace(base, sig_r=np.stack([d.sig_r for d in per_e]), sig_l=np.stack([d.sig_l for d in per_e]),
                              sig_g=np.stack([d.sig_g for d in per_e]))
    other = w.scattering_self_energies(w.random_device(4, 5, 7, overlap=0.05), 30, norm=0.05)
    E2 = well_posed(other, np.linspace(-1.0, 1.0, 7))[:3]
    p = HostProblem(nb, dev, E, sc_stride=4 * 5 * 5)
    q = HostProblem(nb, other, E2)
    out, info = _run_rgf(L, nb, [q, p], opts=nb.make_options(batch=2))
    assert np.all(info == 0)
    names = ("GR_diag", "GL_diag", "GG_upper")
    for prob, devs, energies, slot in ((p, per_e, E, 1), (q, [other] * E2.size, E2, 0)):
        for k, e in enumerate(energies):
            ref, tol = point_tolerance(
                lambda: orgf.solve_point(devs[k], e, 1e-8, 0.1, -0.1, 0.025, greater=True), names, base=1e-11)
            for name, ref_name, diag in (("GRd", "GR_diag", 1), ("GLd", "GL_diag", 1), ("GGu", "GG_upper", 0)):
                got = _unpack(out[name], [q, p], diag)[slot][k]
                assert rel(got, getattr(ref, ref_name)) < tol[ref_name], (name, slot, k)
    # a stride shorter than one energy's blocks is rejected
    bad = HostProblem(nb, dev, E, sc_stride=4 * 5 * 5 - 1)
    arr = (nb.negf_problem * 1)(bad.s)
    assert L.negf_workspace_bytes(nb.OP_LESSER_GREATER, arr, 1, 0, None) == 0


@pytest.mark.parametrize("prec,tol", [(1, 1e-6), (2, 1e-2)])
def test_hostsim_chosen_forms(sim, prec, tol):
    L, nb = sim
    dev = w.slab_device(4, 24, 2)
    E = np.array([0.2])
    p = HostProblem(nb, dev, E)
    out, info = _run_rgf(L, nb, [p], prec=prec, greater=False)
    ref = orgf.solve_point(dev, 0.2, 1e-8, 0.1, -0.1, 0.025)
    e_r = rel(_unpack(out["GRd"], [p], 1)[0][0], ref.GR_diag)
    e_l = rel(_unpack(out["GLd"], [p], 1)[0][0], ref.GL_diag)
    assert e_r < tol and e_l < tol
    if prec == 1:
        assert e_r < 1e-8


def test_hostsim_coupling_slab_maps(sim):
    """b = 128 slab: the products that take a coupling block skip its zero
    16 x 64 slabs.  The test double rejects a map that marks a nonzero slab as
    zero (wrong block or operand), and the results equal the dense ones."""
    L, nb = sim
    dev = w.slab_device(3, 128, 2)
    E = np.array([0.3])
    p = HostProblem(nb, dev, E)
    sparse, info_s = _run_rgf(L, nb, [p], greater=False)
    dense, info_d = _run_rgf(L, nb, [p], greater=False, opts=nb.make_options(dense_coupling=1))
    assert np.all(info_s == info_d)
    for k in ("GRd", "GRu", "GRl", "GLd", "GLu"):
        assert np.array_equal(sparse[k], dense[k]), k
    ref, tol = point_tolerance(lambda: orgf.solve_point(dev, 0.3, 1e-8, 0.1, -0.1, 0.025), ["GR_diag"])
    assert rel(_unpack(sparse["GRd"], [p], 1)[0][0], ref.GR_diag) < tol["GR_diag"]


def test_hostsim_empty_energy_list(sim):
    """A problem with no energies contributes no points; the others are unchanged."""
    L, nb = sim
    dev = w.random_device(3, 4, 7, overlap=0.05)
    E = well_posed(dev, np.linspace(-1.2, 1.2, 9))[:2]
    empty = HostProblem(nb, dev, np.array([]))
    full = HostProblem(nb, dev, E)
    both, info_b = _run_rgf(L, nb, [empty, full], greater=False)
    alone, info_a = _run_rgf(L, nb, [full], greater=False)
    assert info_b.size == 2 and np.array_equal(info_b, info_a)
    for k in ("GRd", "GRu", "GRl", "GLd", "GLu"):
        assert np.array_equal(both[k], alone[k]), k


def test_hostsim_mixed_shapes_and_chunking(sim):
    L, nb = sim
    devs = [w.random_device(3, 4, 11), w.random_device(4, 6, 12, overlap=0.05), w.random_device(3, 4, 13)]
    ens = [well_posed(d, np.linspace(-1.2, 1.2, 9))[:k] for d, k in zip(devs, (3, 1, 2))]
    probs = [HostProblem(nb, d, e) for d, e in zip(devs, ens)]
    full, _ = _run_rgf(L, nb, probs, greater=False)
    chunked, _ = _run_rgf(L, nb, probs, greater=False, opts=nb.make_options(batch=2))
    for name in ("GRd", "GLu"):
        assert np.array_equal(full[name], chunked[name])
    for q, (d, e) in enumerate(zip(devs, ens)):
        got = _unpack(full["GLd"], probs, 1)[q]
        for k, E in enumerate(e):
            ref = orgf.solve_point(d, E, 1e-8, 0.1, -0.1, 0.025)
            assert rel(got[k], ref.GL_diag) < 1e-11


def test_hostsim_transmission_and_obc(sim):
    L, nb = sim
    dev = w.random_device(6, 4, 1)
    E = np.array([-0.8, 0.1, 1.2])
    p = HostProblem(nb, dev, E, eta=1e-6)
    arr = (nb.negf_problem * 1)(p.s)
    ws = np.zeros(L.negf_workspace_bytes(nb.OP_TRANSMISSION, arr, 1, 0, None) + 256, dtype=np.uint8)
    T = np.zeros(3)
    info = np.zeros(3, dtype=np.int32)
    assert L.negf_transmission(arr, 1, None, T.ctypes.data, info.ctypes.data, ws.ctypes.data, ws.size, None) == 0
    for k, e in enumerate(E):
        ref = orgf.solve_point(dev, e, 1e-6, lesser_greater=False, want_T=True).T
        assert abs(T[k] - ref) < 1e-11
    for side in (0, 1):
        ws = np.zeros(L.negf_workspace_bytes(nb.OP_OBC, arr, 1, 0, None) + 256, dtype=np.uint8)
        g = np.zeros((3, 4, 4), complex)
        s = np.zeros((3, 4, 4), complex)
        it = np.zeros(3, np.int32)
        res = np.zeros(3)
        assert L.negf_obc_surface(arr, 1, side, None, None, g.ctypes.data, s.ctypes.data, it.ctypes.data,
                                  res.ctypes.data, info.ctypes.data, ws.ctypes.data, ws.size, None) == 0
        for k, e in enumerate(E):
            r = oleads.lead_self_energy(dev, side, e, 1e-6)
            assert rel(g[k], r.g_surf) < 1e-11 and rel(s[k], r.sigma_r) < 1e-11
            assert it[k] == r.iters
        assert np.all(info == 0) and np.all(res < 1e-10)


def test_hostsim_seeded_obc(sim):
    """An exact seed is accepted with zero iterations; a poor one runs the
    decimation, closed with the seed after every step (as the oracle does)."""
    L, nb = sim
    dev = w.random_device(3, 4, 2)
    E = np.array([0.3, -0.6])
    p = HostProblem(nb, dev, E)
    arr = (nb.negf_problem * 1)(p.s)
    exact = np.stack([oleads.lead_self_energy(dev, 0, e, 1e-8).g_surf for e in E])
    seed = exact.copy()
    seed[1] = np.eye(4) * 0.3                       # a poor guess for the second point
    ws = np.zeros(L.negf_workspace_bytes(nb.OP_OBC, arr, 1, 0, None) + 256, dtype=np.uint8)
    g = np.zeros((2, 4, 4), complex)
    s = np.zeros((2, 4, 4), complex)
    it = np.zeros(2, np.int32)
    res = np.zeros(2)
    info = np.zeros(2, np.int32)
    assert L.negf_obc_surface(arr, 1, 0, None, seed.ctypes.data, g.ctypes.data, s.ctypes.data, it.ctypes.data,
                              res.ctypes.data, info.ctypes.data, ws.ctypes.data, ws.size, None) == 0
    # the oracle's seeded solve decides the path: candidate, closure after step k, or plain
    for k, e in enumerate(E):
        d, a, c = oleads.lead_blocks(dev, 0, e, 1e-8)
        g_ref, k_ref, how = oleads.seeded_sancho_rubio(d, a, c, seed[k])
        assert (how == "candidate") == (k == 0)
        assert abs(int(it[k]) - k_ref) <= 1, (k, int(it[k]), k_ref, how)
        # the closure is accepted at a Dyson residual <= 1e-8, so it sits within
        # ~1e-8 of the converged decimation; the same steps on both sides agree closely
        assert rel(g[k], exact[k]) < 1e-7 and rel(g[k], g_ref) < 1e-11
    assert it[0] == 0 and it[1] > 0
    assert np.all(info == 0)


def test_hostsim_noconv_and_singular_info(sim):
    L, nb = sim
    dev = w.random_device(3, 4, 2)
    p = HostProblem(nb, dev, np.array([0.3]))
    out, info = _run_rgf(L, nb, [p], opts=nb.make_options(sr_max_iter=1), greater=False)
    assert info[0] == nb.NEGF_ENOCONV


def test_hostsim_plan_matches_plain_calls(sim):
    """The plan (fixed decimation count, chunks over worker streams) gives the
    same blocks as the plain call, eagerly and through the graph path.  The
    simulation runs kernels when they are enqueued, so the chunks run while the
    per-stream graphs are captured and a later replay runs only the fork and
    join on the caller's stream (which rewrites the start stamp)."""
    L, nb = sim
    devs = [w.random_device(3, 4, 21), w.random_device(4, 6, 22, overlap=0.05), w.random_device(5, 4, 23)]
    ens = [well_posed(d, np.linspace(-1.2, 1.2, 9))[:k] for d, k in zip(devs, (3, 2, 3))]
    probs = [HostProblem(nb, d, e) for d, e in zip(devs, ens)]
    ref, ref_info = _run_rgf(L, nb, probs, greater=False)
    arr = (nb.negf_problem * len(probs))(*[p.s for p in probs])
    tun = (C.c_int32 * 10)(4, 0, 0, 16, 2, 6, 0, 0, 32, 1)   # (b, tile, tile_f32, inv_nb, batch) for b = 4, 6
    plan = C.c_void_p()
    assert L.negf_plan_create(arr, len(probs), 0, None, C.cast(tun, C.c_void_p), 2, 3, C.byref(plan)) == 0
    nch = L.negf_plan_chunks(plan, None, None, None)
    fp = (C.c_int32 * nch)()
    npn = (C.c_int32 * nch)()
    si = (C.c_int32 * nch)()
    L.negf_plan_chunks(plan, fp, npn, si)
    assert sum(npn) == sum(p.n for p in probs) and max(npn) <= 2 and set(si) <= {0, 1, 2}
    ws = np.zeros(L.negf_plan_workspace_bytes(plan), dtype=np.uint8)
    nd = sum(p.n * p.nb * p.b * p.b for p in probs)
    nu = sum(p.n * (p.nb - 1) * p.b * p.b for p in probs)
    out = {k: np.zeros(nd if k.endswith("d") else nu, dtype=np.complex128) for k in ("GRd", "GRu", "GRl", "GLd", "GLu")}
    info = np.zeros(sum(p.n for p in probs), dtype=np.int32)
    stamps = np.zeros(nch + 1, dtype=np.uint64)
    for run, use_graph in enumerate((0, 1, 1)):
        assert L.negf_plan_execute(plan, use_graph, out["GRd"].ctypes.data, out["GRu"].ctypes.data,
                                   out["GRl"].ctypes.data, out["GLd"].ctypes.data, out["GLu"].ctypes.data, None, None,
                                   info.ctypes.data, stamps.ctypes.data, ws.ctypes.data, ws.size, None) == 0
        assert np.array_equal(info, ref_info)
        for k in out:
            assert rel(out[k], ref[k]) < 1e-13, k
        if run < 2:
            assert np.all(stamps[1:] > stamps[0])
    L.negf_plan_destroy(plan)


def test_hostsim_point_queue_rounds_and_results(sim):
    """negf_plan_run_queue (eager) on the CPU double: three problems of two shapes
    (the first two share one chunk) with 7, 5 and 4 tasks over 3, 2 and 4 slots
    (3, 3 and 1 rounds, partial last rounds), two worker streams.  Every task's density of states matches the
    oracle's at its energy, info is clear, every task is stamped, and the task
    counts are reached exactly (no task solved twice or skipped)."""
    L, nb = sim
    vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    L.negf_plan_queue_bytes.argtypes = [vp]
    L.negf_plan_queue_bytes.restype = sz
    L.negf_plan_run_queue.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp,
                                      sz, vp]
    devs = [w.random_device(10, 8, 1), w.random_device(10, 8, 2), w.slab_device(6, 12, 7)]
    slots = [3, 2, 4]
    tasks = [np.linspace(-2.1, 2.2, 7), np.array([-1.3, -0.6, 0.1, 0.9, 1.4]), np.array([-2.5, -0.2, 0.8, 2.3])]
    probs = [HostProblem(nb, d, np.zeros(n), eta=1e-6) for d, n in zip(devs, slots)]
    arr = (nb.negf_problem * 3)(*[p.s for p in probs])
    plan = C.c_void_p()
    assert L.negf_plan_create(arr, 3, 0, None, None, 0, 2, C.byref(plan)) == 0
    ws = np.zeros(L.negf_plan_workspace_bytes(plan) + 256, dtype=np.uint8)
    qws = np.zeros(L.negf_plan_queue_bytes(plan) + 256, dtype=np.uint8)
    nd = sum(p.n * p.nb * p.b * p.b for p in probs)
    nu = sum(p.n * (p.nb - 1) * p.b * p.b for p in probs)
    out = {k: np.zeros(nd if k.endswith("d") else nu, dtype=np.complex128) for k in ("GRd", "GRu", "GRl", "GLd", "GLu")}
    info = np.zeros(sum(slots), dtype=np.int32)
    tE = [np.ascontiguousarray(t) for t in tasks]
    total = sum(t.size for t in tE)
    t_info = np.full(total, -7, dtype=np.int32)
    t_dos = np.zeros(total)
    t_stamp = np.zeros(total, dtype=np.uint64)
    start = np.zeros(1, dtype=np.uint64)
    ptrs = (C.c_void_p * 3)(*[t.ctypes.data for t in tE])
    counts = (C.c_int32 * 3)(*[t.size for t in tE])
    d = lambda k: out[k].ctypes.data
    code = L.negf_plan_run_queue(plan, 0, ptrs, counts, t_info.ctypes.data, t_dos.ctypes.data, t_stamp.ctypes.data,
                                 start.ctypes.data, d("GRd"), d("GRu"), d("GRl"), d("GLd"), d("GLu"), None, None,
                                 info.ctypes.data, qws.ctypes.data, qws.size, ws.ctypes.data, ws.size, None)
    assert code == 0
    L.negf_plan_destroy(plan)
    assert np.all(t_info == 0), t_info
    assert np.all(t_stamp > start[0]), (t_stamp, start)
    off = 0
    for dev, t in zip(devs, tE):
        for i, E in enumerate(t):
            ref = orgf.solve_point(dev, float(E), 1e-6, 0.1, -0.1, 0.025, lesser_greater=False)
            dos_ref = -np.imag(sum(np.trace(g) for g in ref.GR_diag)) / np.pi
            assert abs(t_dos[off + i] - dos_ref) <= 1e-9 * abs(dos_ref) + 1e-12, (E, t_dos[off + i], dos_ref)
        off += t.size
    # the last round's slots: problem 0 ran tasks 6 (slot 0) and nothing new in slots 1, 2
    assert probs[0].E[0] == tE[0][6] and probs[0].E[1] == tE[0][4] and probs[0].E[2] == tE[0][5]
