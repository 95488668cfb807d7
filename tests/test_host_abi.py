"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments synchronously (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "negf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(negf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2602_03438_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2602_03438_amd import build
        build.build()
    return binding.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("negf_obc_surface", "negf_rgf_retarded", "negf_rgf_lesser_greater", "negf_transmission",
                 "negf_workspace_bytes", "negf_status_string", "negf_version"):
        assert must in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_version(L):
    from paper_2602_03438_amd import binding as nb
    assert nb.status_string(nb.NEGF_OK) == "ok"
    assert "converge" in nb.status_string(nb.NEGF_ENOCONV)
    assert nb.negf_version() >= nb.ABI_VERSION == 102


def _fake_problem(nb_=4, b=8, n_e=3, h=True):
    from paper_2602_03438_amd import binding as nbd
    # host addresses stand in for device pointers: nothing is dereferenced on these paths
    buf = np.zeros(16, dtype=np.complex128)
    p = buf.ctypes.data
    dev = nbd.negf_device(nb_, b, p if h else None, p if h else None, None, None, None, None, None)
    return nbd.negf_problem(dev, n_e, p, 1e-8, 0.1, -0.1, 0.025), buf


def test_workspace_bytes_host_logic(L):
    from paper_2602_03438_amd import binding as nb
    pr, keep = _fake_problem()
    arr = (nb.negf_problem * 1)(pr)
    n_r = L.negf_workspace_bytes(nb.OP_RETARDED, arr, 1, nb.PLAIN_FP64, None)
    n_l = L.negf_workspace_bytes(nb.OP_LESSER_GREATER, arr, 1, nb.PLAIN_FP64, None)
    n_ref = L.negf_workspace_bytes(nb.OP_LESSER_GREATER, arr, 1, nb.FP32_REFINE, None)
    assert 0 < n_r <= n_l < n_ref
    # the batch option bounds the points in flight
    opt = nb.make_options(batch=1)
    assert L.negf_workspace_bytes(nb.OP_RETARDED, arr, 1, nb.PLAIN_FP64, C.byref(opt)) < n_r
    bad, keep2 = _fake_problem(nb_=1)
    assert L.negf_workspace_bytes(nb.OP_RETARDED, (nb.negf_problem * 1)(bad), 1, 0, None) == 0
    bad, keep3 = _fake_problem(h=False)
    assert L.negf_workspace_bytes(nb.OP_RETARDED, (nb.negf_problem * 1)(bad), 1, 0, None) == 0
    bad, keep4 = _fake_problem(b=2048)
    assert L.negf_workspace_bytes(nb.OP_RETARDED, (nb.negf_problem * 1)(bad), 1, 0, None) == 0


def test_invalid_arguments_return_einval_synchronously(L):
    from paper_2602_03438_amd import binding as nb
    pr, keep = _fake_problem()
    arr = (nb.negf_problem * 1)(pr)
    # null outputs / workspace / zero problems: rejected before any device work
    assert L.negf_rgf_retarded(arr, 1, 0, None, None, None, None, None, None, 0, None) == nb.NEGF_EINVAL
    assert L.negf_rgf_retarded(arr, 0, 0, None, None, None, None, None, None, 0, None) == nb.NEGF_EINVAL
    assert L.negf_rgf_lesser_greater(arr, 1, 0, None, None, None, None, None, None, None, None, None, None, 0,
                                     None) == nb.NEGF_EINVAL
    assert L.negf_transmission(arr, 1, None, None, None, None, 0, None) == nb.NEGF_EINVAL
    assert L.negf_obc_surface(arr, 1, 2, None, None, None, None, None, None, None, None, 0, None) == nb.NEGF_EINVAL
    # a workspace that is too small
    x = np.zeros(64, dtype=np.complex128)
    p = x.ctypes.data
    info = np.zeros(3, dtype=np.int32)
    assert L.negf_rgf_retarded(arr, 1, 0, None, p, p, None, info.ctypes.data, p, 16, None) == nb.NEGF_EINVAL
    # misaligned output pointer
    assert L.negf_rgf_retarded(arr, 1, 0, None, p + 8, p, None, info.ctypes.data, p, 1 << 40, None) == nb.NEGF_EINVAL
    # bad precision code
    assert L.negf_rgf_retarded(arr, 1, 7, None, p, p, None, info.ctypes.data, p, 1 << 40, None) == nb.NEGF_EINVAL
    # kernel-level entry points
    one = (C.c_double * 2)(1.0, 0.0)
    assert L.negf_zgemm_batched(b"X", b"N", 4, 4, 4, one, p, 4, 16, p, 4, 16, one, p, 4, 16, 1, 0, 0,
                                None) == nb.NEGF_EINVAL
    assert L.negf_zinv_batched(2048, 1, p, p + 16, None, 16, p, 1 << 30, None) == nb.NEGF_EINVAL
    assert L.negf_zinv_batched(4, 1, p, p, None, 16, p, 1 << 30, None) == nb.NEGF_EINVAL


def test_static_entry_point_rejects_synchronously(L):
    """negf_rgf_lesser_greater_static: argument errors and a point that does not
    fit the static scratch return before anything touches a GPU (the pointers
    below are never dereferenced)."""
    from paper_2602_03438_amd import binding as nb
    fake = C.c_void_p(1 << 20)
    dev = nb.negf_device(60, 512, fake, fake, None, None, None, None, None)
    arr = (nb.negf_problem * 1)(nb.negf_problem(dev, 1, fake, 1e-8, 0.0, 0.0, 0.025))
    outs = [fake] * 7
    st = L.negf_rgf_lesser_greater_static(arr, 1, nb.PLAIN_FP64, None, *outs, fake, None)
    assert st == nb.NEGF_ENOMEM          # ~368 MiB of workspace per point > 256 MiB of scratch
    st = L.negf_rgf_lesser_greater_static(arr, 1, nb.PLAIN_FP64, None, *outs, None, None)
    assert st == nb.NEGF_EINVAL          # info is required
    small = nb.negf_device(60, 128, fake, fake, None, None, None, None, None)
    arr2 = (nb.negf_problem * 1)(nb.negf_problem(small, 12, fake, 1e-8, 0.0, 0.0, 0.025))
    st = L.negf_rgf_lesser_greater_static(arr2, 1, nb.PLAIN_FP64, C.byref(nb.make_options(batch=12)), *outs, fake,
                                          None)
    assert st == nb.NEGF_ENOMEM          # 12 points in flight need ~283 MiB
    assert L.negf_workspace_bytes(nb.OP_LESSER_GREATER, arr2, 1, nb.PLAIN_FP64, None) > (256 << 20)


def test_energy_convolution_and_transpose_reject_synchronously(L):
    """negf_energy_convolution / negf_transpose: sizes, the FFT length limit, overlap,
    alignment and workspace are checked before anything is enqueued; empty inputs
    return OK without touching the GPU."""
    from paper_2602_03438_amd import binding as nb
    buf = np.zeros(64, dtype=np.complex128)
    p = buf.ctypes.data
    one = (C.c_double * 2)(1.0, 0.0)
    assert L.negf_econv_workspace_bytes(1024, 1024) == 2048 * 16 + 256
    assert L.negf_econv_workspace_bytes(5, 3) == 16 * 16 + 256          # L at least 16
    assert L.negf_econv_workspace_bytes(3000, 1200) == 0                # n_e + n_w - 1 > 4096
    assert L.negf_econv_workspace_bytes(0, 5) == 0
    ws = L.negf_econv_workspace_bytes(8, 4)
    G, W, B = p, p + 256, p + 512
    ok_args = lambda **k: dict(dict(n_e=8, n_el=2, G=G, n_w=4, k0=1, W=W, scale=one, B=B, ws=p, ws_bytes=ws), **k)
    call = lambda a: L.negf_energy_convolution(a["n_e"], a["n_el"], a["G"], a["n_w"], a["k0"], a["W"], a["scale"],
                                               a["B"], a["ws"], a["ws_bytes"], None)
    assert call(ok_args(n_el=0)) == nb.NEGF_OK                          # nothing to do
    for bad in (dict(n_e=0), dict(n_w=0), dict(k0=4), dict(k0=-1), dict(n_el=-1), dict(B=G), dict(B=W),
                dict(G=G + 8), dict(ws_bytes=ws - 1), dict(ws=None), dict(scale=None), dict(n_el=1 << 31),
                dict(n_e=3000, n_w=1200, k0=0)):
        assert call(ok_args(**bad)) == nb.NEGF_EINVAL, bad
    assert L.negf_transpose(0, 5, p, p + 256, None) == nb.NEGF_OK
    assert L.negf_transpose(-1, 5, p, p + 256, None) == nb.NEGF_EINVAL
    assert L.negf_transpose(3, 5, p, p, None) == nb.NEGF_EINVAL
    assert L.negf_transpose(3, 5, p + 8, p + 256, None) == nb.NEGF_EINVAL


def test_partitioned_inversion_layout_and_rejects(L):
    """negf_serinv_workspace_bytes is 0 for a partition count the block count cannot
    hold (fewer than 2 partitions, periods below 3 blocks, an empty last partition),
    and the call rejects those layouts and missing outputs synchronously."""
    from paper_2602_03438_amd import binding as nb
    pr, keep = _fake_problem(nb_=14, b=8, n_e=2)
    arr = (nb.negf_problem * 1)(pr)
    for parts, ok in ((1, False), (2, True), (3, True), (4, True), (5, True), (6, False), (14, False)):
        n = L.negf_serinv_workspace_bytes(arr, parts, 0)
        assert (n > 0) == ok, (parts, n)
    assert L.negf_serinv_workspace_bytes(arr, 3, 1) > L.negf_serinv_workspace_bytes(arr, 3, 0)
    p = keep.ctypes.data
    ws = L.negf_serinv_workspace_bytes(arr, 3, 0)
    info = np.zeros(2, dtype=np.int32).ctypes.data
    call = lambda parts, grd=p, wsb=ws, inf=info: L.negf_serinv_lesser_greater(
        arr, parts, None, grd, p, p, p, p, None, None, inf, p, wsb, None)
    assert call(1) == nb.NEGF_EINVAL
    assert call(6) == nb.NEGF_EINVAL
    assert call(3, grd=None) == nb.NEGF_EINVAL
    assert call(3, inf=None) == nb.NEGF_EINVAL
    assert call(3, wsb=ws - 1) == nb.NEGF_EINVAL


def test_point_queue_rejects_synchronously(L):
    from paper_2602_03438_amd import binding as nb
    assert L.negf_plan_queue_bytes(None) == 0
    p = np.zeros(8, dtype=np.complex128).ctypes.data
    assert L.negf_plan_run_queue(None, 0, None, None, None, None, None, None, p, p, p, p, p, None, None, p, p, 1024,
                                 p, 1024, None) == nb.NEGF_EINVAL


def test_self_consistent_loop_rejects_synchronously(L):
    """negf_scba: a device that already carries scattering self-energies, an out-of-range bath
    index, mixing, Anderson memory, tolerance or iteration cap, a convolution longer than 4096,
    missing or aliased buffers and a short workspace all return EINVAL before any work."""
    from paper_2602_03438_amd import binding as nb
    pr, keep = _fake_problem(nb_=4, b=8, n_e=6)
    arr = (nb.negf_problem * 1)(pr)
    n_w = 5
    ws = L.negf_scba_workspace_bytes(arr, 1, nb.PLAIN_FP64, None, n_w, 0)
    sig_bytes = 6 * 4 * 8 * 8 * 16
    assert ws >= L.negf_workspace_bytes(nb.OP_LESSER_GREATER, arr, 1, nb.PLAIN_FP64, None) + 2 * sig_bytes
    assert L.negf_scba_workspace_bytes(arr, 1, nb.PLAIN_FP64, None, 0, 0) == 0
    assert L.negf_scba_workspace_bytes(arr, 1, nb.PLAIN_FP64, None, 4092, 0) == 0   # 6 + 4092 - 1 > 4096
    assert L.negf_scba_workspace_bytes(arr, 0, nb.PLAIN_FP64, None, n_w, 0) == 0
    # Anderson memory 1..4: room for 2 M + 2 history vectors of both kinds; beyond 4 rejected
    ws3 = L.negf_scba_workspace_bytes(arr, 1, nb.PLAIN_FP64, None, n_w, 3)
    assert ws3 >= ws + 8 * 2 * sig_bytes
    assert L.negf_scba_workspace_bytes(arr, 1, nb.PLAIN_FP64, None, n_w, 5) == 0
    assert L.negf_scba_workspace_bytes(arr, 1, nb.PLAIN_FP64, None, n_w, -1) == 0
    # k-points must share the block shape and the energy count; several need room for their average
    other, keep_o = _fake_problem(nb_=4, b=8, n_e=5)
    assert L.negf_scba_workspace_bytes((nb.negf_problem * 2)(pr, other), 2, nb.PLAIN_FP64, None, n_w, 0) == 0
    two = L.negf_scba_workspace_bytes((nb.negf_problem * 2)(pr, pr), 2, nb.PLAIN_FP64, None, n_w, 0)
    assert two > ws
    one = (C.c_double * 2)(0.0, 1.0)
    bufs = [np.zeros(64, dtype=np.complex128) for _ in range(13)]
    W_l, W_g, s_r, s_l, s_g, grd, gru, grl, gld, glu, ggd, ggu, info = [b.ctypes.data for b in bufs]
    n_iter = C.c_int32(-1)
    hist = (C.c_double * 8)()

    def call(a=arr, k0=2, mixing=0.5, memory=0, tol=1e-10, max_iter=8, wsb=ws, **over):
        p = dict(W_l=W_l, W_g=W_g, s_r=s_r, s_l=s_l, s_g=s_g, ggd=ggd, info=info, scale=one, n_iter=C.byref(n_iter))
        p.update(over)
        return L.negf_scba(a, 1, nb.PLAIN_FP64, None, n_w, k0, p["W_l"], p["W_g"], p["scale"], mixing, memory, tol, max_iter,
                           p["s_r"], p["s_l"], p["s_g"], grd, gru, grl, gld, glu, p["ggd"], ggu, p["info"],
                           p["n_iter"], hist, grd, wsb, None)

    for bad in (dict(k0=-1), dict(k0=5), dict(mixing=0.0), dict(mixing=1.5), dict(mixing=float("nan")),
                dict(tol=-1.0), dict(max_iter=0), dict(wsb=ws - 1), dict(W_l=None), dict(ggd=None), dict(info=None),
                dict(scale=None), dict(n_iter=None), dict(s_l=s_g), dict(W_g=W_g + 8), dict(memory=5),
                dict(memory=-1), dict(memory=3)):   # memory 3 needs the larger workspace
        assert call(**bad) == nb.NEGF_EINVAL, bad
    # the loop supplies the scattering self-energies: a device with its own is rejected
    dev = nb.negf_device(4, 8, W_l, W_l, None, None, s_r, s_l, s_g)
    with_sc = (nb.negf_problem * 1)(nb.negf_problem(dev, 6, W_l, 1e-8, 0.1, -0.1, 0.025))
    assert call(a=with_sc) == nb.NEGF_EINVAL
    strided = (nb.negf_problem * 1)(nb.negf_problem(pr.dev, 6, W_l, 1e-8, 0.1, -0.1, 0.025, 4 * 8 * 8))
    assert call(a=strided) == nb.NEGF_EINVAL


def test_self_consistent_step_rejects_synchronously(L):
    """negf_scba_step: the checks of negf_scba plus a negative iteration index and a missing state."""
    from paper_2602_03438_amd import binding as nb
    pr, keep = _fake_problem(nb_=4, b=8, n_e=6)
    arr = (nb.negf_problem * 1)(pr)
    ws = L.negf_scba_workspace_bytes(arr, 1, nb.PLAIN_FP64, None, 5, 0)
    one = (C.c_double * 2)(0.0, 1.0)
    bufs = [np.zeros(64, dtype=np.complex128) for _ in range(14)]
    W_l, W_g, s_r, s_l, s_g, grd, gru, grl, gld, glu, ggd, ggu, info, state = [b.ctypes.data for b in bufs]

    def call(it=0, st=state, k0=2, wsb=ws, memory=0):
        return L.negf_scba_step(arr, 1, nb.PLAIN_FP64, None, 5, k0, W_l, W_g, one, 0.5, memory, 1e-10, it, 1, s_r, s_l, s_g, grd,
                                gru, grl, gld, glu, ggd, ggu, info, None, st, grd, wsb, None)
    assert call(it=-1) == nb.NEGF_EINVAL
    assert call(st=None) == nb.NEGF_EINVAL
    assert call(k0=5) == nb.NEGF_EINVAL
    assert call(wsb=ws - 1) == nb.NEGF_EINVAL
    assert call(memory=5) == nb.NEGF_EINVAL
    assert call(memory=1) == nb.NEGF_EINVAL     # workspace sized for linear mixing


def test_observables_reject_synchronously(L):
    """negf_observables: an output without the Green's function it needs, misalignment, more than
    65535 energies in a problem; nothing requested is a no-op."""
    from paper_2602_03438_amd import binding as nb
    pr, keep = _fake_problem(nb_=4, b=8, n_e=3)
    arr = (nb.negf_problem * 1)(pr)
    x = np.zeros(64, dtype=np.complex128)
    p = x.ctypes.data
    assert L.negf_observables(arr, 1, None, None, None, None, None) == nb.NEGF_OK
    assert L.negf_observables(arr, 1, None, p, p, None, None) == nb.NEGF_EINVAL      # dos needs GR_diag
    assert L.negf_observables(arr, 1, p, None, None, p, None) == nb.NEGF_EINVAL      # current needs GL_upper
    assert L.negf_observables(arr, 1, p + 8, p, p, p, None) == nb.NEGF_EINVAL
    assert L.negf_observables(arr, 0, p, p, p, p, None) == nb.NEGF_EINVAL
    big, keep2 = _fake_problem(nb_=4, b=8, n_e=70000)
    assert L.negf_observables((nb.negf_problem * 1)(big), 1, p, p, p, p, None) == nb.NEGF_EINVAL
