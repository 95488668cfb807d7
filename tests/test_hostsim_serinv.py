"""The partitioned selected inversion (negf_serinv_lesser_greater), run on the
CPU through the host test double of the kernels, against the oracle: every
partition count and layout (middle partitions present or not, last partition
shorter than the others), with S != I and scattering self-energies, G^R, G^<
and G^>."""
import ctypes as C
import os

import numpy as np
import pytest

import workloads as w
from helpers import plain_reference
from oracle import rgf as orgf

HERE = os.path.dirname(os.path.abspath(__file__))
NAMES = ["GR_diag", "GR_upper", "GR_lower", "GL_diag", "GL_upper", "GG_diag", "GG_upper"]


@pytest.fixture(scope="module")
def sim():
    from paper_2602_03438_amd import binding as nb
    import importlib.util
    spec = importlib.util.spec_from_file_location("hostsim_build", os.path.join(HERE, "hostsim", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    L = C.CDLL(mod.build(sanitize=os.environ.get("NEGF_HOSTSIM_SANITIZED") == "1"))
    P = C.POINTER
    vp, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    L.negf_serinv_workspace_bytes.argtypes = [P(nb.negf_problem), i32, i32]
    L.negf_serinv_workspace_bytes.restype = sz
    L.negf_serinv_lesser_greater.argtypes = [P(nb.negf_problem), i32, P(nb.negf_options), vp, vp, vp, vp, vp, vp, vp,
                                             vp, vp, sz, vp]
    return L, nb


def _run(L, nb, dev, energies, parts, eta=1e-6):
    keep = [np.ascontiguousarray(x) if x is not None else None
            for x in (dev.H_diag, dev.H_upper, dev.S_diag, dev.S_upper, dev.sig_r, dev.sig_l, dev.sig_g)]
    E = np.ascontiguousarray(energies, dtype=np.float64)
    ptr = lambda a: a.ctypes.data if a is not None else None
    d = nb.negf_device(dev.nb, dev.b, *[ptr(a) for a in keep])
    prob = (nb.negf_problem * 1)(nb.negf_problem(d, E.size, E.ctypes.data, eta, 0.1, -0.1, 0.025))
    nbytes = L.negf_serinv_workspace_bytes(prob, parts, 1)
    assert nbytes > 0
    ws = np.zeros(nbytes, dtype=np.uint8)
    n, b, nbk = E.size, dev.b, dev.nb
    out = {k: np.full((n, nbk if k.endswith("diag") else nbk - 1, b, b), np.nan, dtype=np.complex128) for k in NAMES}
    info = np.zeros(n, dtype=np.int32)
    code = L.negf_serinv_lesser_greater(prob, parts, None, *[out[k].ctypes.data for k in NAMES], info.ctypes.data,
                                        ws.ctypes.data, ws.size, None)
    assert code == 0, code
    return out, info


@pytest.mark.parametrize("nbk,parts", [(6, 2), (9, 2), (11, 3), (14, 4), (13, 4), (21, 5), (22, 5), (17, 3), (60, 8)])
def test_serinv_matches_oracle(sim, nbk, parts):
    L, nb = sim
    dev = w.random_device(nbk, 4, 7 + nbk, overlap=0.05)
    w.scattering_self_energies(dev, 5, norm=0.05)
    energies = np.array([-0.55, 0.4])
    out, info = _run(L, nb, dev, energies, parts)
    assert np.all(info == 0)
    for k, E in enumerate(energies):
        ref, _ = plain_reference(lambda: orgf.solve_point(dev, E, 1e-6, 0.1, -0.1, 0.025, greater=True), NAMES)
        for name in NAMES:
            err = np.linalg.norm(out[name][k] - getattr(ref, name)) / np.linalg.norm(getattr(ref, name))
            assert err <= 1e-10, (nbk, parts, E, name, err)


def test_serinv_rejects_layouts_it_cannot_form(sim):
    L, nb = sim
    dev = w.random_device(6, 3, 1)
    keep = [np.ascontiguousarray(dev.H_diag), np.ascontiguousarray(dev.H_upper)]
    E = np.array([0.1])
    d = nb.negf_device(6, 3, keep[0].ctypes.data, keep[1].ctypes.data, None, None, None, None, None)
    prob = (nb.negf_problem * 1)(nb.negf_problem(d, 1, E.ctypes.data, 1e-6, 0.0, 0.0, 0.025))
    assert L.negf_serinv_workspace_bytes(prob, 1, 0) == 0       # one partition is not a partitioning
    assert L.negf_serinv_workspace_bytes(prob, 3, 0) == 0       # period 3 leaves no last interior
    assert L.negf_serinv_workspace_bytes(prob, 2, 0) > 0
