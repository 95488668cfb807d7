"""ctypes binding of libnegf.so (see include/negf.h for the contract).

The functions named ``negf_*`` are the C entry points with argument
marshalling only.  The helpers below them (``DeviceOnGPU``, ``Problem``,
``obc_surface``, ``rgf_retarded``, ``rgf_lesser_greater``, ``transmission``,
``zgemm``, ``zinv``) allocate outputs and workspace as torch tensors on the
current HIP device and pass raw pointers and the current stream.  Every
number is computed by the library's HIP kernels; there is no fallback path:
if libnegf.so is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnegf.so")

NEGF_OK, NEGF_EINVAL, NEGF_ENOCONV, NEGF_ESINGULAR, NEGF_ENONFINITE, NEGF_EHIP, NEGF_ENOMEM = range(7)
ABI_VERSION = 102          # negf_version() of the struct layouts and loop signatures below
PLAIN_FP64, FP32_REFINE, FP32_NOREFINE = 0, 1, 2
OP_OBC, OP_RETARDED, OP_LESSER_GREATER, OP_TRANSMISSION = 0, 1, 2, 3
KC_NAMES = ["gemm_f64", "gemm_f32", "inv_panel", "inv_swap", "inv_perm", "elementwise", "inv_update_gemm",
            "gemm_coupling"]
KC_COUNT = 8


class negf_device(C.Structure):
    _fields_ = [("nb", C.c_int32), ("b", C.c_int32),
                ("H_diag", C.c_void_p), ("H_upper", C.c_void_p),
                ("S_diag", C.c_void_p), ("S_upper", C.c_void_p),
                ("sig_r_sc", C.c_void_p), ("sig_l_sc", C.c_void_p), ("sig_g_sc", C.c_void_p)]


class negf_problem(C.Structure):
    _fields_ = [("dev", negf_device), ("n_e", C.c_int32), ("energies", C.c_void_p),
                ("eta", C.c_double), ("mu_l", C.c_double), ("mu_r", C.c_double), ("kT", C.c_double),
                ("sc_stride", C.c_int64)]


class negf_options(C.Structure):
    _fields_ = [("sr_tol", C.c_double), ("sr_max_iter", C.c_int32), ("sr_accept", C.c_double),
                ("batch", C.c_int32), ("inv_nb", C.c_int32), ("xcd_remap", C.c_int32), ("gemm_tile", C.c_int32),
                ("gemm_tile_f32", C.c_int32), ("cmul", C.c_int32), ("dense_coupling", C.c_int32)]


class negf_tuning(C.Structure):
    _fields_ = [("b", C.c_int32), ("gemm_tile", C.c_int32), ("gemm_tile_f32", C.c_int32), ("inv_nb", C.c_int32),
                ("batch", C.c_int32)]


class negf_kernel_stats(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("flops", C.c_double), ("bytes", C.c_double)]


class NegfError(RuntimeError):
    pass


_lib = None


def lib():
    """Load libnegf.so once; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise NegfError(f"{LIB_PATH} is missing: build it with `python -m paper_2602_03438_amd.build`")
    L = C.CDLL(LIB_PATH)
    P = C.POINTER
    vp, i32, i64, sz, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t, C.c_double
    L.negf_workspace_bytes.argtypes = [i32, P(negf_problem), i32, i32, P(negf_options)]
    L.negf_workspace_bytes.restype = sz
    L.negf_obc_surface.argtypes = [P(negf_problem), i32, i32, P(negf_options), vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.negf_obc_surface.restype = C.c_int
    L.negf_rgf_retarded.argtypes = [P(negf_problem), i32, i32, P(negf_options), vp, vp, vp, vp, vp, sz, vp]
    L.negf_rgf_retarded.restype = C.c_int
    L.negf_rgf_lesser_greater.argtypes = [P(negf_problem), i32, i32, P(negf_options), vp, vp, vp, vp, vp, vp, vp,
                                          vp, vp, sz, vp]
    L.negf_rgf_lesser_greater.restype = C.c_int
    L.negf_rgf_lesser_greater_static.argtypes = [P(negf_problem), i32, i32, P(negf_options), vp, vp, vp, vp, vp,
                                                 vp, vp, vp, vp]
    L.negf_rgf_lesser_greater_static.restype = C.c_int
    L.negf_serinv_workspace_bytes.argtypes = [P(negf_problem), i32, i32]
    L.negf_serinv_workspace_bytes.restype = sz
    L.negf_serinv_lesser_greater.argtypes = [P(negf_problem), i32, P(negf_options), vp, vp, vp, vp, vp, vp, vp, vp,
                                             vp, sz, vp]
    L.negf_serinv_lesser_greater.restype = C.c_int
    L.negf_econv_workspace_bytes.argtypes = [i32, i32]
    L.negf_econv_workspace_bytes.restype = sz
    L.negf_energy_convolution.argtypes = [i32, i64, vp, i32, i32, vp, P(dbl), vp, vp, sz, vp]
    L.negf_energy_convolution.restype = C.c_int
    L.negf_transpose.argtypes = [i64, i64, vp, vp, vp]
    L.negf_transpose.restype = C.c_int
    L.negf_scba_workspace_bytes.argtypes = [P(negf_problem), i32, i32, P(negf_options), i32, i32]
    L.negf_scba_workspace_bytes.restype = sz
    L.negf_scba.argtypes = [P(negf_problem), i32, i32, P(negf_options), i32, i32, vp, vp, P(dbl), dbl, i32, dbl, i32,
                            vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, P(i32), P(dbl), vp, sz, vp]
    L.negf_scba.restype = C.c_int
    L.negf_scba_step.argtypes = [P(negf_problem), i32, i32, P(negf_options), i32, i32, vp, vp, P(dbl), dbl, i32, dbl,
                                 i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.negf_scba_step.restype = C.c_int
    L.negf_observables.argtypes = [P(negf_problem), i32, vp, vp, vp, vp, vp]
    L.negf_observables.restype = C.c_int
    L.negf_transmission.argtypes = [P(negf_problem), i32, P(negf_options), vp, vp, vp, sz, vp]
    L.negf_transmission.restype = C.c_int
    L.negf_zgemm_batched.argtypes = [C.c_char, C.c_char, i32, i32, i32, P(dbl), vp, i64, i64, vp, i64, i64, P(dbl),
                                     vp, i64, i64, i32, i32, i32, vp]
    L.negf_zgemm_batched.restype = C.c_int
    L.negf_inverse_workspace_bytes.argtypes = [i32, i32]
    L.negf_inverse_workspace_bytes.restype = sz
    L.negf_zinv_batched.argtypes = [i32, i32, vp, vp, vp, i32, vp, sz, vp]
    L.negf_zinv_batched.restype = C.c_int
    L.negf_profile_enable.argtypes = [i32]
    L.negf_profile_enable.restype = None
    L.negf_profile_time_classes.argtypes = [C.c_uint32]
    L.negf_profile_time_classes.restype = None
    L.negf_profile_read.argtypes = [P(negf_kernel_stats)]
    L.negf_profile_read.restype = C.c_int
    L.negf_status_string.argtypes = [C.c_int]
    L.negf_status_string.restype = C.c_char_p
    L.negf_version.argtypes = []
    L.negf_version.restype = i32
    L.negf_plan_create.argtypes = [P(negf_problem), i32, i32, P(negf_options), P(negf_tuning), i32, i32, P(vp)]
    L.negf_plan_create.restype = C.c_int
    L.negf_plan_workspace_bytes.argtypes = [vp]
    L.negf_plan_workspace_bytes.restype = sz
    L.negf_plan_chunks.argtypes = [vp, vp, vp, vp]
    L.negf_plan_chunks.restype = i32
    L.negf_plan_execute.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.negf_plan_execute.restype = C.c_int
    L.negf_plan_queue_bytes.argtypes = [vp]
    L.negf_plan_queue_bytes.restype = sz
    L.negf_plan_run_queue.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp, sz,
                                      vp]
    L.negf_plan_run_queue.restype = C.c_int
    L.negf_plan_clock_hz.argtypes = []
    L.negf_plan_clock_hz.restype = dbl
    L.negf_plan_destroy.argtypes = [vp]
    L.negf_plan_destroy.restype = None
    if hasattr(L, "negf_mlp_forward"):
        _bind_mlp(L)
    if L.negf_version() < ABI_VERSION:
        raise NegfError(f"{LIB_PATH} is older than this binding (negf_problem layout {L.negf_version()}, "
                        f"need {ABI_VERSION}): rebuild it")
    _lib = L
    return L


def _bind_mlp(L):
    vp, i32, sz, flt = C.c_void_p, C.c_int32, C.c_size_t, C.c_float
    L.negf_mlp_forward.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.negf_mlp_forward.restype = C.c_int
    L.negf_mlp_backward.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                    vp]
    L.negf_mlp_backward.restype = C.c_int
    L.negf_mlp_adam_step.argtypes = [i32, vp, vp, vp, vp, i32, flt, flt, flt, flt, vp]
    L.negf_mlp_adam_step.restype = C.c_int
    L.negf_mlp_infer_bf16.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.negf_mlp_infer_bf16.restype = C.c_int
    L.negf_mlp_to_bf16.argtypes = [vp, vp, C.c_int64, vp]
    L.negf_mlp_to_bf16.restype = C.c_int
    i64 = C.c_int64
    L.negf_mlp_moments.argtypes = [i64, i32, vp, vp, vp, vp, vp]
    L.negf_mlp_moments.restype = C.c_int
    L.negf_mlp_normalize.argtypes = [i64, i32, vp, vp, vp, vp, vp]
    L.negf_mlp_normalize.restype = C.c_int
    L.negf_mlp_signed_log.argtypes = [i64, vp, vp, i32, vp]
    L.negf_mlp_signed_log.restype = C.c_int
    L.negf_mlp_mse.argtypes = [i64, vp, vp, vp, vp, vp]
    L.negf_mlp_mse.restype = C.c_int
    L.negf_mode_diag.argtypes = [i32, i32, vp, vp, vp]
    L.negf_mode_diag.restype = C.c_int
    L.negf_mode_scale_columns.argtypes = [i32, i32, vp, vp, vp, vp]
    L.negf_mode_scale_columns.restype = C.c_int


def status_string(code: int) -> str:
    return lib().negf_status_string(code).decode()


def check(code: int, what: str = "negf call"):
    if code != NEGF_OK:
        raise NegfError(f"{what} failed: {status_string(code)} ({code})")


# ---------------------------------------------------------------- raw entry points

def negf_workspace_bytes(op, problems, n_prob, prec, opt):
    return lib().negf_workspace_bytes(op, problems, n_prob, prec, opt)


def negf_obc_surface(*args):
    return lib().negf_obc_surface(*args)


def negf_rgf_retarded(*args):
    return lib().negf_rgf_retarded(*args)


def negf_rgf_lesser_greater(*args):
    return lib().negf_rgf_lesser_greater(*args)


def negf_rgf_lesser_greater_static(*args):
    return lib().negf_rgf_lesser_greater_static(*args)


def negf_serinv_workspace_bytes(*args):
    return lib().negf_serinv_workspace_bytes(*args)


def negf_serinv_lesser_greater(*args):
    return lib().negf_serinv_lesser_greater(*args)


def negf_transmission(*args):
    return lib().negf_transmission(*args)


def negf_zgemm_batched(*args):
    return lib().negf_zgemm_batched(*args)


def negf_zinv_batched(*args):
    return lib().negf_zinv_batched(*args)


def negf_inverse_workspace_bytes(n, batch):
    return lib().negf_inverse_workspace_bytes(n, batch)


def negf_profile_enable(on):
    lib().negf_profile_enable(int(on))


def negf_profile_time_classes(mask):
    lib().negf_profile_time_classes(int(mask) & 0xFFFFFFFF)


def negf_profile_read():
    arr = (negf_kernel_stats * KC_COUNT)()
    check(lib().negf_profile_read(arr), "negf_profile_read")
    return {KC_NAMES[i]: dict(launches=arr[i].launches, total_ms=arr[i].total_ms, flops=arr[i].flops,
                              bytes=arr[i].bytes) for i in range(KC_COUNT)}


def negf_version():
    return lib().negf_version()


# ---------------------------------------------------------------- torch helpers

def _torch():
    import torch
    if not torch.cuda.is_available():
        raise NegfError("no HIP device available: libnegf.so runs on the GPU only")
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def to_gpu(a: Optional[np.ndarray]):
    if a is None:
        return None
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


class DeviceOnGPU:
    """The blocks of one block-tridiagonal device resident in HBM."""

    def __init__(self, dev):
        self.nb = dev.nb
        self.b = dev.b
        self.H_diag = to_gpu(dev.H_diag)
        self.H_upper = to_gpu(dev.H_upper)
        self.S_diag = to_gpu(dev.S_diag)
        self.S_upper = to_gpu(dev.S_upper)
        self.sig_r = to_gpu(dev.sig_r)
        self.sig_l = to_gpu(dev.sig_l)
        self.sig_g = to_gpu(dev.sig_g)

    def struct(self) -> negf_device:
        return negf_device(self.nb, self.b, _ptr(self.H_diag), _ptr(self.H_upper), _ptr(self.S_diag),
                           _ptr(self.S_upper), _ptr(self.sig_r), _ptr(self.sig_l), _ptr(self.sig_g))


class Problem:
    """A device on the GPU plus its energies and contact parameters."""

    def __init__(self, dev: DeviceOnGPU, energies, eta=1e-8, mu_l=0.0, mu_r=0.0, kT=0.025, sc_stride=0):
        """``sc_stride`` > 0: the device's scattering self-energies are [n_e][nb][b][b], one set per
        energy, ``sc_stride`` elements apart (normally nb b b)."""
        torch = _torch()
        self.dev = dev
        self.energies = torch.as_tensor(np.asarray(energies, dtype=np.float64)).to("cuda")
        self.eta, self.mu_l, self.mu_r, self.kT = float(eta), float(mu_l), float(mu_r), float(kT)
        self.sc_stride = int(sc_stride)

    @property
    def n_e(self):
        return int(self.energies.numel())

    def struct(self) -> negf_problem:
        return negf_problem(self.dev.struct(), self.n_e, _ptr(self.energies), self.eta, self.mu_l, self.mu_r, self.kT,
                            self.sc_stride)


def _problem_array(problems: Sequence[Problem]):
    arr = (negf_problem * len(problems))(*[p.struct() for p in problems])
    return arr


def make_options(sr_tol=0.0, sr_max_iter=0, sr_accept=0.0, batch=0, inv_nb=0, xcd_remap=-1, gemm_tile=0,
                 gemm_tile_f32=0, cmul=0, dense_coupling=0):
    """negf_options; 0 (or -1 for xcd_remap) leaves a knob at the library default.
    cmul: real products per complex double product, 4 or 3 (Gauss's method).
    dense_coupling: 1 multiplies the coupling blocks as dense blocks (no skipping
    of their zero slabs)."""
    return negf_options(sr_tol, sr_max_iter, sr_accept, batch, inv_nb, xcd_remap, gemm_tile, gemm_tile_f32, cmul,
                        dense_coupling)


def _alloc_blocks(problems, per_point_blocks):
    torch = _torch()
    tot = sum(p.n_e * per_point_blocks(p) * p.dev.b * p.dev.b for p in problems)
    return torch.empty(tot, dtype=torch.complex128, device="cuda")


def _split(flat, problems, per_point_blocks):
    out, off = [], 0
    for p in problems:
        n = p.n_e * per_point_blocks(p) * p.dev.b * p.dev.b
        out.append(flat[off:off + n].view(p.n_e, per_point_blocks(p), p.dev.b, p.dev.b))
        off += n
    return out


class Workspace:
    """Reusable device workspace (a torch uint8 buffer)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes):
        torch = _torch()
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        return self.buf


def workspace_bytes(op, problems, prec=PLAIN_FP64, opts=None):
    arr = _problem_array(problems)
    return negf_workspace_bytes(op, arr, len(problems), prec, C.byref(opts) if opts else None)


def obc_surface(problems: List[Problem], side: int, opts=None, seed=None, ws: Optional[Workspace] = None):
    torch = _torch()
    if seed is not None and not seed.is_contiguous():
        raise NegfError("seed must be a C-contiguous [points, b, b] complex128 tensor")
    arr = _problem_array(problems)
    o = C.byref(opts) if opts else None
    nbytes = negf_workspace_bytes(OP_OBC, arr, len(problems), PLAIN_FP64, o)
    if nbytes == 0:
        raise NegfError("invalid problems")
    buf = (ws or Workspace()).get(nbytes)
    one = lambda p: 1
    g = _alloc_blocks(problems, one)
    sig = _alloc_blocks(problems, one)
    npts = sum(p.n_e for p in problems)
    iters = torch.zeros(npts, dtype=torch.int32, device="cuda")
    resid = torch.zeros(npts, dtype=torch.float64, device="cuda")
    info = torch.zeros(npts, dtype=torch.int32, device="cuda")
    code = negf_obc_surface(arr, len(problems), side, o, _ptr(seed), _ptr(g), _ptr(sig), _ptr(iters), _ptr(resid),
                            _ptr(info), _ptr(buf), buf.numel(), _stream())
    check(code, "negf_obc_surface")
    return dict(g_surf=_split(g, problems, one), sigma_r=_split(sig, problems, one), iters=iters, resid=resid,
                info=info)


def _rgf_outputs(problems, lesser, greater, lower):
    diag = lambda p: p.dev.nb
    off = lambda p: p.dev.nb - 1
    out = dict(GR_diag=_alloc_blocks(problems, diag), GR_upper=_alloc_blocks(problems, off),
               GR_lower=_alloc_blocks(problems, off) if lower else None)
    if lesser:
        out["GL_diag"] = _alloc_blocks(problems, diag)
        out["GL_upper"] = _alloc_blocks(problems, off)
    if greater:
        out["GG_diag"] = _alloc_blocks(problems, diag)
        out["GG_upper"] = _alloc_blocks(problems, off)
    return out


def _check_outputs(out, problems, lesser, greater, lower):
    """Caller-supplied outputs: every required array a contiguous complex128 device tensor
    with room for all points (the library writes through raw pointers)."""
    torch = _torch()
    need_d = sum(p.n_e * p.dev.nb * p.dev.b * p.dev.b for p in problems)
    need_o = sum(p.n_e * (p.dev.nb - 1) * p.dev.b * p.dev.b for p in problems)
    req = {"GR_diag": need_d, "GR_upper": need_o}
    if lower:
        req["GR_lower"] = need_o
    if lesser:
        req.update(GL_diag=need_d, GL_upper=need_o)
    if greater:
        req.update(GG_diag=need_d, GG_upper=need_o)
    for k, n in req.items():
        v = out.get(k)
        if v is None or not v.is_cuda or v.dtype != torch.complex128 or not v.is_contiguous() or v.numel() < n:
            raise NegfError(f"outputs[{k!r}] must be a contiguous complex128 device tensor of at least {n} elements")
    return out


def _views(flat, problems):
    res = {}
    for k, v in flat.items():
        if v is None:
            res[k] = None
            continue
        per = (lambda p: p.dev.nb) if k.endswith("diag") else (lambda p: p.dev.nb - 1)
        res[k] = _split(v, problems, per)
    return res


def rgf_retarded(problems, prec=PLAIN_FP64, opts=None, lower=True, ws=None, outputs=None):
    torch = _torch()
    arr = _problem_array(problems)
    o = C.byref(opts) if opts else None
    nbytes = negf_workspace_bytes(OP_RETARDED, arr, len(problems), prec, o)
    if nbytes == 0:
        raise NegfError("invalid problems")
    buf = (ws or Workspace()).get(nbytes)
    out = _check_outputs(outputs, problems, False, False, lower) if outputs else _rgf_outputs(problems, False, False, lower)
    npts = sum(p.n_e for p in problems)
    info = torch.zeros(npts, dtype=torch.int32, device="cuda")
    code = negf_rgf_retarded(arr, len(problems), prec, o, _ptr(out["GR_diag"]), _ptr(out["GR_upper"]),
                             _ptr(out.get("GR_lower")), _ptr(info), _ptr(buf), buf.numel(), _stream())
    check(code, "negf_rgf_retarded")
    res = _views(out, problems)
    res["info"] = info
    res["flat"] = out
    return res


def rgf_lesser_greater(problems, prec=PLAIN_FP64, opts=None, greater=False, lower=True, ws=None, outputs=None):
    torch = _torch()
    arr = _problem_array(problems)
    o = C.byref(opts) if opts else None
    nbytes = negf_workspace_bytes(OP_LESSER_GREATER, arr, len(problems), prec, o)
    if nbytes == 0:
        raise NegfError("invalid problems")
    buf = (ws or Workspace()).get(nbytes)
    out = _check_outputs(outputs, problems, True, greater, lower) if outputs else _rgf_outputs(problems, True, greater, lower)
    npts = sum(p.n_e for p in problems)
    info = torch.zeros(npts, dtype=torch.int32, device="cuda")
    code = negf_rgf_lesser_greater(arr, len(problems), prec, o, _ptr(out["GR_diag"]), _ptr(out["GR_upper"]),
                                   _ptr(out.get("GR_lower")), _ptr(out["GL_diag"]), _ptr(out["GL_upper"]),
                                   _ptr(out.get("GG_diag")), _ptr(out.get("GG_upper")), _ptr(info), _ptr(buf),
                                   buf.numel(), _stream())
    check(code, "negf_rgf_lesser_greater")
    res = _views(out, problems)
    res["info"] = info
    res["flat"] = out
    return res


def rgf_lesser_greater_static(problems, prec=PLAIN_FP64, opts=None, greater=False, lower=True, outputs=None):
    """negf_rgf_lesser_greater_static: the library's own static scratch instead of a
    workspace.  Outputs (and info) are allocated here unless given; the call itself
    allocates nothing.  Returns the raw status next to the outputs (NEGF_ENOMEM
    when a point does not fit the scratch) instead of raising."""
    torch = _torch()
    arr = _problem_array(problems)
    o = C.byref(opts) if opts else None
    out = _check_outputs(outputs, problems, True, greater, lower) if outputs else _rgf_outputs(problems, True, greater, lower)
    npts = sum(p.n_e for p in problems)
    info = torch.zeros(npts, dtype=torch.int32, device="cuda")
    code = negf_rgf_lesser_greater_static(arr, len(problems), prec, o, _ptr(out["GR_diag"]), _ptr(out["GR_upper"]),
                                          _ptr(out.get("GR_lower")), _ptr(out["GL_diag"]), _ptr(out["GL_upper"]),
                                          _ptr(out.get("GG_diag")), _ptr(out.get("GG_upper")), _ptr(info), _stream())
    res = _views(out, problems)
    res["info"] = info
    res["flat"] = out
    res["status"] = code
    return res


def serinv_lesser_greater(problem, partitions, opts=None, greater=False, lower=True, ws=None, outputs=None):
    """negf_serinv_lesser_greater for one problem: the partitioned selected inversion
    (same outputs as rgf_lesser_greater)."""
    torch = _torch()
    arr = _problem_array([problem])
    nbytes = negf_serinv_workspace_bytes(arr, partitions, int(greater))
    if nbytes == 0:
        raise NegfError("invalid problem or partition count for the partitioned inversion")
    buf = (ws or Workspace()).get(nbytes)
    out = _check_outputs(outputs, [problem], True, greater, lower) if outputs else _rgf_outputs([problem], True, greater, lower)
    info = torch.zeros(problem.n_e, dtype=torch.int32, device="cuda")
    code = negf_serinv_lesser_greater(arr, partitions, C.byref(opts) if opts else None, _ptr(out["GR_diag"]),
                                      _ptr(out["GR_upper"]), _ptr(out.get("GR_lower")), _ptr(out["GL_diag"]),
                                      _ptr(out["GL_upper"]), _ptr(out.get("GG_diag")), _ptr(out.get("GG_upper")),
                                      _ptr(info), _ptr(buf), buf.numel(), _stream())
    check(code, "negf_serinv_lesser_greater")
    res = _views(out, [problem])
    res["info"] = info
    res["flat"] = out
    return res


def energy_convolution(G, W, k0, scale=1.0, out=None, ws=None):
    """negf_energy_convolution of energy-major complex128 tensors G [n_e, n_el] and
    W [n_w, n_el]: B[e] = scale * sum_k G[e + k0 - k] * W[k]."""
    torch = _torch()
    for t in (G, W):
        if not t.is_contiguous() or t.dtype != torch.complex128 or t.dim() != 2:
            raise NegfError("G and W must be C-contiguous 2-D complex128 tensors [energies, elements]")
    n_e, n_el = G.shape
    n_w = W.shape[0]
    if W.shape[1] != n_el:
        raise NegfError("G and W must have the same number of elements")
    nbytes = lib().negf_econv_workspace_bytes(n_e, n_w)
    if nbytes == 0:
        raise NegfError("n_e + n_w - 1 exceeds the longest transform (4096)")
    buf = (ws or Workspace()).get(nbytes)
    B = out if out is not None else torch.empty_like(G)
    if not B.is_contiguous() or B.dtype != torch.complex128 or tuple(B.shape) != (n_e, n_el) or not B.is_cuda:
        raise NegfError("out must be a C-contiguous complex128 device tensor of G's shape")
    sc = (C.c_double * 2)(complex(scale).real, complex(scale).imag)
    check(lib().negf_energy_convolution(n_e, n_el, _ptr(G), n_w, int(k0), _ptr(W), sc, _ptr(B), _ptr(buf),
                                        buf.numel(), _stream()), "negf_energy_convolution")
    return B


def scba(problem, W_lesser, W_greater, k0, scale, mixing=0.5, tol=1e-10, max_iter=50, sig0=None, prec=PLAIN_FP64,
         opts=None, lower=True, ws=None, outputs=None, sigmas=None, memory=0):
    """negf_scba: the self-consistent loop of Fig. 1 with a fixed bath, for one problem or a list of
    problems (one per k-point, same block shape and energies; the outputs and info then run over
    them in order, point-major, and the self-energies are shared).

    W_lesser / W_greater: complex128 device tensors [n_w, nb, b, b] (W[k] at (k - k0) dE);
    scale: the convolution's prefactor (e.g. 1j dE / 2 pi); memory: 0 for linear mixing, 1..4 for
    Anderson mixing over that many previous iterations; sig0: optional (Sigma^<, Sigma^>)
    [n_e, nb, b, b] to start from (default zero); sigmas: optional dict of caller-owned
    sig_r / sig_l / sig_g tensors to run in place (their lesser / greater contents are the
    start when sig0 is None).  Returns the outputs (per-point views), the final self-energies,
    info, n_iter, the residual history and the status (OK: converged; ENOCONV: max_iter reached;
    ENONFINITE: a non-finite residual)."""
    torch = _torch()
    probs = list(problem) if isinstance(problem, (list, tuple)) else [problem]
    arr = _problem_array(probs)
    o = C.byref(opts) if opts else None
    dv = probs[0].dev
    n_w = int(W_lesser.shape[0])
    shape = (probs[0].n_e, dv.nb, dv.b, dv.b)
    for t in (W_lesser, W_greater):
        if (not t.is_cuda or t.dtype != torch.complex128 or not t.is_contiguous()
                or tuple(t.shape) != (n_w, dv.nb, dv.b, dv.b)):
            raise NegfError("W_lesser / W_greater must be contiguous complex128 device tensors [n_w, nb, b, b]")
    nbytes = lib().negf_scba_workspace_bytes(arr, len(probs), prec, o, n_w, int(memory))
    if nbytes == 0:
        raise NegfError("invalid problem or bath for the self-consistent loop")
    buf = (ws or Workspace()).get(nbytes)
    if sigmas is None:
        sigmas = {k: torch.zeros(shape, dtype=torch.complex128, device="cuda") for k in ("sig_r", "sig_l", "sig_g")}
    for k in ("sig_r", "sig_l", "sig_g"):
        t = sigmas.get(k)
        if t is None or not t.is_cuda or t.dtype != torch.complex128 or not t.is_contiguous() or tuple(t.shape) != shape:
            raise NegfError(f"sigmas[{k!r}] must be a contiguous complex128 device tensor {shape}")
    if sig0 is not None:
        sigmas["sig_l"].copy_(torch.as_tensor(sig0[0]).to(sigmas["sig_l"].device))
        sigmas["sig_g"].copy_(torch.as_tensor(sig0[1]).to(sigmas["sig_g"].device))
    out = (_check_outputs(outputs, probs, True, True, lower) if outputs
           else _rgf_outputs(probs, True, True, lower))
    info = torch.zeros(sum(p.n_e for p in probs), dtype=torch.int32, device="cuda")
    sc = (C.c_double * 2)(complex(scale).real, complex(scale).imag)
    n_iter = C.c_int32(0)
    hist = (C.c_double * max(int(max_iter), 1))()
    code = lib().negf_scba(arr, len(probs), prec, o, n_w, int(k0), _ptr(W_lesser), _ptr(W_greater), sc, float(mixing), int(memory),
                           float(tol), int(max_iter), _ptr(sigmas["sig_r"]), _ptr(sigmas["sig_l"]), _ptr(sigmas["sig_g"]),
                           _ptr(out["GR_diag"]), _ptr(out["GR_upper"]), _ptr(out.get("GR_lower")),
                           _ptr(out["GL_diag"]), _ptr(out["GL_upper"]), _ptr(out["GG_diag"]), _ptr(out["GG_upper"]),
                           _ptr(info), C.byref(n_iter), hist, _ptr(buf), buf.numel(), _stream())
    if code not in (NEGF_OK, NEGF_ENOCONV, NEGF_ENONFINITE):
        check(code, "negf_scba")
    res = _views(out, probs)
    res.update(sigmas)
    res["info"] = info
    res["flat"] = out
    res["n_iter"] = int(n_iter.value)
    res["history"] = [hist[i] for i in range(n_iter.value)]
    res["status"] = int(code)
    return res


def observables(problems, outputs, dos=True, current=True):
    """negf_observables on the flat outputs of rgf_lesser_greater (or rgf_retarded, for dos alone):
    returns {"dos": [per problem: (n_e, nb)], "current": [per problem: (n_e, nb - 1)]} float64 device
    tensors."""
    torch = _torch()
    arr = _problem_array(problems)
    nd = sum(p.n_e * p.dev.nb for p in problems)
    nc = sum(p.n_e * (p.dev.nb - 1) for p in problems)
    D = torch.empty(max(1, nd), dtype=torch.float64, device="cuda") if dos else None
    J = torch.empty(max(1, nc), dtype=torch.float64, device="cuda") if current else None
    check(lib().negf_observables(arr, len(problems), _ptr(outputs.get("GR_diag")) if dos else None,
                                 _ptr(outputs.get("GL_upper")) if current else None, _ptr(D), _ptr(J), _stream()),
          "negf_observables")
    res, od, oc = {"dos": [], "current": []}, 0, 0
    for p in problems:
        if dos:
            res["dos"].append(D[od:od + p.n_e * p.dev.nb].view(p.n_e, p.dev.nb))
        if current:
            res["current"].append(J[oc:oc + p.n_e * (p.dev.nb - 1)].view(p.n_e, p.dev.nb - 1))
        od += p.n_e * p.dev.nb
        oc += p.n_e * (p.dev.nb - 1)
    return res


class ScbaLoop:
    """The loop of negf_scba as single steps (negf_scba_step): nothing synchronises, so a run of
    steps can be captured in a graph.  Holds the self-energies, the outputs, the per-point info,
    the device history and the device state {solves, 0 running / 1 converged / 2 non-finite}."""

    def __init__(self, problem, W_lesser, W_greater, k0, scale, mixing=0.5, tol=1e-10, max_steps=64,
                 prec=PLAIN_FP64, opts=None, lower=True, memory=0):
        torch = _torch()
        self.problems = list(problem) if isinstance(problem, (list, tuple)) else [problem]
        self.problem, self.Wl, self.Wg, self.k0 = self.problems[0], W_lesser, W_greater, int(k0)
        self.scale = (C.c_double * 2)(complex(scale).real, complex(scale).imag)
        self.mixing, self.tol, self.prec, self.opts = float(mixing), float(tol), prec, opts
        self.memory = int(memory)
        self._arr = _problem_array(self.problems)
        dv = self.problem.dev
        self.n_w = int(W_lesser.shape[0])
        for t in (W_lesser, W_greater):
            if (not t.is_cuda or t.dtype != torch.complex128 or not t.is_contiguous()
                    or tuple(t.shape) != (self.n_w, dv.nb, dv.b, dv.b)):
                raise NegfError("W_lesser / W_greater must be contiguous complex128 device tensors [n_w, nb, b, b]")
        o = C.byref(opts) if opts else None
        nbytes = lib().negf_scba_workspace_bytes(self._arr, len(self.problems), prec, o, self.n_w, self.memory)
        if nbytes == 0:
            raise NegfError("invalid problem or bath for the self-consistent loop")
        self.ws = Workspace().get(nbytes)
        shape = (self.problem.n_e, dv.nb, dv.b, dv.b)
        self.sig = {k: torch.zeros(shape, dtype=torch.complex128, device="cuda") for k in ("sig_r", "sig_l", "sig_g")}
        self.out = _rgf_outputs(self.problems, True, True, lower)
        self.info = torch.zeros(sum(p.n_e for p in self.problems), dtype=torch.int32, device="cuda")
        self.history = torch.zeros(max(1, int(max_steps)), dtype=torch.float64, device="cuda")
        self.state = torch.zeros(2, dtype=torch.int32, device="cuda")

    def step(self, it, update=True):
        if not 0 <= it < self.history.numel():
            raise NegfError("iteration index beyond the history")
        o = self.out
        check(lib().negf_scba_step(self._arr, len(self.problems), self.prec, C.byref(self.opts) if self.opts else None, self.n_w, self.k0,
                                   _ptr(self.Wl), _ptr(self.Wg), self.scale, self.mixing, self.memory, self.tol, int(it),
                                   int(bool(update)), _ptr(self.sig["sig_r"]), _ptr(self.sig["sig_l"]),
                                   _ptr(self.sig["sig_g"]), _ptr(o["GR_diag"]), _ptr(o["GR_upper"]),
                                   _ptr(o.get("GR_lower")), _ptr(o["GL_diag"]), _ptr(o["GL_upper"]),
                                   _ptr(o["GG_diag"]), _ptr(o["GG_upper"]), _ptr(self.info), _ptr(self.history),
                                   _ptr(self.state), _ptr(self.ws), self.ws.numel(), _stream()), "negf_scba_step")

    def run(self, n):
        """n steps, the last without mixing."""
        for it in range(n):
            self.step(it, update=it < n - 1)


def transpose(X, out=None):
    """negf_transpose of a C-contiguous 2-D complex128 tensor."""
    torch = _torch()
    if not X.is_contiguous() or X.dtype != torch.complex128 or X.dim() != 2:
        raise NegfError("transpose needs a C-contiguous 2-D complex128 tensor")
    r, c = X.shape
    Y = out if out is not None else torch.empty(c, r, dtype=X.dtype, device=X.device)
    if not Y.is_contiguous() or Y.dtype != torch.complex128 or tuple(Y.shape) != (c, r) or not Y.is_cuda:
        raise NegfError("out must be a C-contiguous complex128 device tensor of the transposed shape")
    check(lib().negf_transpose(r, c, _ptr(X), _ptr(Y), _stream()), "negf_transpose")
    return Y


def transmission(problems, opts=None, ws=None):
    torch = _torch()
    arr = _problem_array(problems)
    o = C.byref(opts) if opts else None
    nbytes = negf_workspace_bytes(OP_TRANSMISSION, arr, len(problems), PLAIN_FP64, o)
    if nbytes == 0:
        raise NegfError("invalid problems")
    buf = (ws or Workspace()).get(nbytes)
    npts = sum(p.n_e for p in problems)
    T = torch.zeros(npts, dtype=torch.float64, device="cuda")
    info = torch.zeros(npts, dtype=torch.int32, device="cuda")
    code = negf_transmission(arr, len(problems), o, _ptr(T), _ptr(info), _ptr(buf), buf.numel(), _stream())
    check(code, "negf_transmission")
    return dict(T=T, info=info)


def zgemm(A, B, C_=None, opa="N", opb="N", alpha=1.0, beta=0.0, prec=0, tile=0):
    """Batched complex product on the library kernel: C = alpha op(A) op(B) + beta C."""
    torch = _torch()
    for t in (A, B, C_):
        if t is not None and not t.is_contiguous():
            raise NegfError("zgemm operands must be C-contiguous [batch, rows, cols] complex128 tensors")
    batch = A.shape[0]
    M = A.shape[1] if opa == "N" else A.shape[2]
    K = A.shape[2] if opa == "N" else A.shape[1]
    N = B.shape[2] if opb == "N" else B.shape[1]
    if C_ is None:
        C_ = torch.zeros(batch, M, N, dtype=torch.complex128, device="cuda")
    al = (C.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (C.c_double * 2)(complex(beta).real, complex(beta).imag)
    code = negf_zgemm_batched(opa.encode(), opb.encode(), M, N, K, al, _ptr(A), A.shape[2], A.shape[1] * A.shape[2],
                              _ptr(B), B.shape[2], B.shape[1] * B.shape[2], be, _ptr(C_), N, M * N, batch, prec, tile,
                              _stream())
    check(code, "negf_zgemm_batched")
    return C_


def zinv(M, nb=32):
    """Batched inverse of [batch, n, n] complex128 blocks (M is copied, not destroyed)."""
    torch = _torch()
    batch, n, _ = M.shape
    work = M.contiguous().clone(memory_format=torch.contiguous_format)
    out = torch.empty_like(M)
    info = torch.zeros(batch, dtype=torch.int32, device="cuda")
    nbytes = negf_inverse_workspace_bytes(n, batch)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    code = negf_zinv_batched(n, batch, _ptr(work), _ptr(out), _ptr(info), nb, _ptr(buf), nbytes, _stream())
    check(code, "negf_zinv_batched")
    return out, info


class Plan:
    """A shape-grouped, stream-scheduled batch of problems (negf_plan_*)."""

    def __init__(self, problems, prec=PLAIN_FP64, opts=None, tunings=None, n_streams=4):
        self.problems = list(problems)
        self._arr = _problem_array(self.problems)
        tun = tunings or []
        self._tun = (negf_tuning * max(1, len(tun)))(*[negf_tuning(*t) for t in tun])
        self.handle = C.c_void_p()
        check(lib().negf_plan_create(self._arr, len(self.problems), prec, C.byref(opts) if opts else None,
                                     self._tun if tun else None, len(tun), n_streams, C.byref(self.handle)),
              "negf_plan_create")
        self.ws = Workspace()

    def chunks(self):
        n = lib().negf_plan_chunks(self.handle, None, None, None)
        fp, npn, si = (C.c_int32 * n)(), (C.c_int32 * n)(), (C.c_int32 * n)()
        lib().negf_plan_chunks(self.handle, fp, npn, si)
        return [(fp[i], npn[i], si[i]) for i in range(n)]

    def _checked(self, outputs, info):
        torch = _torch()
        _check_outputs(outputs, self.problems, True, outputs.get("GG_diag") is not None,
                       outputs.get("GR_lower") is not None)
        npts = sum(p.n_e for p in self.problems)
        if info is None or info.dtype != torch.int32 or not info.is_cuda or info.numel() < npts:
            raise NegfError(f"info must be an int32 device tensor of at least {npts} entries")
        return outputs

    def execute(self, outputs, info, use_graph=True, stamps=None):
        buf = self.ws.get(lib().negf_plan_workspace_bytes(self.handle))
        o = self._checked(outputs, info)
        if stamps is not None and (stamps.dtype != _torch().int64 or not stamps.is_cuda or
                                   stamps.numel() < len(self.chunks()) + 1):
            raise NegfError("stamps must be an int64 device tensor of (chunks + 1) entries")
        check(lib().negf_plan_execute(self.handle, int(use_graph), _ptr(o["GR_diag"]), _ptr(o["GR_upper"]),
                                      _ptr(o.get("GR_lower")), _ptr(o["GL_diag"]), _ptr(o["GL_upper"]),
                                      _ptr(o.get("GG_diag")), _ptr(o.get("GG_upper")), _ptr(info), _ptr(stamps),
                                      _ptr(buf), buf.numel(), _stream()), "negf_plan_execute")

    def run_queue(self, task_energies, outputs, info, use_graph=True, results=None):
        """Stream per-problem task lists (device float64 tensors, one per problem)
        through the plan (negf_plan_run_queue).  Returns the task results, each
        concatenated over the problems: info (int32), dos (float64), stamps (int64
        wall-clock ticks), and the start stamp (a one-element int64 tensor); pass
        `results` (a dict from an earlier call) to reuse their buffers."""
        torch = _torch()
        if len(task_energies) != len(self.problems):
            raise NegfError("run_queue: one task list per problem")
        n_tasks = [int(t.numel()) for t in task_energies]
        total = sum(n_tasks)
        if results is None:
            results = {"info": torch.zeros(max(1, total), dtype=torch.int32, device="cuda"),
                       "dos": torch.zeros(max(1, total), dtype=torch.float64, device="cuda"),
                       "stamps": torch.zeros(max(1, total), dtype=torch.int64, device="cuda"),
                       "start": torch.zeros(1, dtype=torch.int64, device="cuda")}
        self._tasks = [t.contiguous() for t in task_energies]
        ptrs = (C.c_void_p * len(self._tasks))(*[_ptr(t) if t.numel() else None for t in self._tasks])
        counts = (C.c_int32 * len(n_tasks))(*n_tasks)
        self._checked(outputs, info)
        buf = self.ws.get(lib().negf_plan_workspace_bytes(self.handle))
        qbytes = lib().negf_plan_queue_bytes(self.handle)
        if getattr(self, "_qws", None) is None or self._qws.numel() < qbytes:
            self._qws = torch.empty(int(qbytes), dtype=torch.uint8, device="cuda")
        o = outputs
        check(lib().negf_plan_run_queue(self.handle, int(use_graph), ptrs, counts, _ptr(results["info"]),
                                        _ptr(results["dos"]), _ptr(results["stamps"]), _ptr(results["start"]),
                                        _ptr(o["GR_diag"]), _ptr(o["GR_upper"]), _ptr(o.get("GR_lower")),
                                        _ptr(o["GL_diag"]), _ptr(o["GL_upper"]), _ptr(o.get("GG_diag")),
                                        _ptr(o.get("GG_upper")), _ptr(info), _ptr(self._qws), self._qws.numel(),
                                        _ptr(buf), buf.numel(), _stream()), "negf_plan_run_queue")
        return results

    def outputs(self, greater=False, lower=True):
        return _rgf_outputs(self.problems, True, greater, lower)

    @staticmethod
    def clock_hz():
        return lib().negf_plan_clock_hz()

    def close(self):
        """Destroy the plan and release its workspace."""
        if self.handle:
            lib().negf_plan_destroy(self.handle)
            self.handle = C.c_void_p()
        self.ws.buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
