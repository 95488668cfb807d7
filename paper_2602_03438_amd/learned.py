"""Learned initial guess for the lead decimation (per-mode MLP).

The paper's outlook (Section IV) proposes machine learning to shortcut
expensive steps of ab-initio transport.  Here a small network proposes the
surface Green's function of a lead from the energy and features of the lead
cell; the decimation checks the proposal by its Dyson residual and falls back
to the plain iteration when it fails (``seed`` argument of negf_obc_surface).

Per-mode model.  A dense b x b complex output cannot come out of a width-256
network, so the guess is built in the generalised eigenbasis of the lead cell,
H0 u_j = lambda_j S0 u_j with U^H S0 U = I (host preprocessing, once per lead):

  features (E, j): E, E - lambda_j, (U^H H1 H1^H U)_jj, (U^H H1^H H1 U)_jj,
                   Re and Im of (U^H H1 U)_jj
  target   x_j   = (U^H S0 g_s S0 U)_jj       (Re, Im)
  seed     g~    = U diag(x) U^H

Training (single precision, Adam, mean squared error) and inference (bf16)
run in the library's MLP kernels; the input standardisation, the signed-log
compression of the targets, the training loss and the mode transforms (the
diagonal of U^H S0 g S0 U, the column scaling U diag(x)) run in the library's
transform kernels and complex product kernel.  torch only holds the memory.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import List

import numpy as np

from . import binding as nb

N_FEAT = 6
WIDTH = 256
N_OUT = 2


@dataclasses.dataclass
class LeadBasis:
    lam: np.ndarray          # [b] generalised eigenvalues of the lead cell
    U: np.ndarray            # [b, b] S0-orthonormal eigenvectors
    feat0: np.ndarray        # [b, 4] energy-independent mode features
    S0: np.ndarray


def lead_basis(dev, side: int = 0) -> LeadBasis:
    """Eigenbasis and mode features of the left (side 0) or right lead of ``dev``."""
    import scipy.linalg as sl
    nb_ = dev.nb
    if side == 0:
        H0, S0 = dev.H_diag[0], dev.s_diag(0)
        H1 = dev.H_upper[0].conj().T
    else:
        H0, S0 = dev.H_diag[nb_ - 1], dev.s_diag(nb_ - 1)
        H1 = dev.H_upper[nb_ - 2]
    lam, U = sl.eigh(H0, S0)
    UH = U.conj().T
    a = np.real(np.einsum("ij,ji->i", UH @ H1, H1.conj().T @ U))
    c = np.real(np.einsum("ij,ji->i", UH @ H1.conj().T, H1 @ U))
    d = np.einsum("ij,ji->i", UH, H1 @ U)
    feat0 = np.stack([a, c, d.real, d.imag], axis=1)
    return LeadBasis(lam, np.ascontiguousarray(U), feat0, S0)


def features(basis: LeadBasis, energies: np.ndarray) -> np.ndarray:
    """[n_e * b, N_FEAT] float32 rows, energy-major."""
    E = np.asarray(energies, dtype=np.float64)
    b = basis.lam.size
    out = np.empty((E.size, b, N_FEAT), dtype=np.float32)
    out[:, :, 0] = E[:, None]
    out[:, :, 1] = E[:, None] - basis.lam[None, :]
    out[:, :, 2:] = basis.feat0[None, :, :]
    return out.reshape(-1, N_FEAT)


class GPUBasis:
    """U, U^H S0 and S0 U of one lead on the GPU, for the target and seed transforms."""

    def __init__(self, basis: LeadBasis):
        import torch
        self.b = basis.lam.size
        U = basis.U
        self.U = torch.from_numpy(U).cuda()
        self.UHS = torch.from_numpy(np.ascontiguousarray(U.conj().T @ basis.S0)).cuda()
        self.SU = torch.from_numpy(np.ascontiguousarray(basis.S0 @ U)).cuda()

    def targets(self, g_surf):
        """x_j = (U^H S0 g S0 U)_jj for a batch [n, b, b] -> float32 [n*b, 2]."""
        import torch
        n = g_surf.shape[0]
        L = self.UHS.unsqueeze(0).expand(n, -1, -1).contiguous()
        R = self.SU.unsqueeze(0).expand(n, -1, -1).contiguous()
        t = nb.zgemm(L, g_surf.contiguous())
        t = nb.zgemm(t, R)
        out = torch.empty(n * self.b, 2, dtype=torch.float32, device="cuda")
        nb.check(nb.lib().negf_mode_diag(n, self.b, nb._ptr(t), nb._ptr(out), nb._stream()), "negf_mode_diag")
        return out

    def seeds(self, y):
        """g~ = U diag(x) U^H from network outputs y [n*b, 2] -> complex128 [n, b, b]."""
        import torch
        n = y.shape[0] // self.b
        y = y.contiguous()
        t = torch.empty(n, self.b, self.b, dtype=torch.complex128, device="cuda")
        nb.check(nb.lib().negf_mode_scale_columns(n, self.b, nb._ptr(self.U), nb._ptr(y), nb._ptr(t), nb._stream()),
                 "negf_mode_scale_columns")
        Ub = self.U.unsqueeze(0).expand(n, -1, -1).contiguous()
        return nb.zgemm(t, Ub, opb="C")


def signed_log(x, inverse=False):
    """sign(x) log(1 + |x|) (or its inverse) of a float32 tensor, in the library's kernel."""
    import torch
    x = x.contiguous()
    y = torch.empty_like(x)
    nb.check(nb.lib().negf_mlp_signed_log(x.numel(), nb._ptr(x), nb._ptr(y), int(inverse), nb._stream()),
             "negf_mlp_signed_log")
    return y


class MLP:
    """Parameters, Adam state and bf16 copies of the per-mode network on the GPU."""

    def __init__(self, seed: int = 0, n_in: int = N_FEAT, width: int = WIDTH, n_out: int = N_OUT):
        import torch
        r = np.random.Generator(np.random.PCG64(seed))
        shapes = [(n_in, width), (width, width), (width, n_out)]
        self.F, self.H, self.O = n_in, width, n_out
        self.p = {}
        for k, (fi, fo) in enumerate(shapes, start=1):
            lim = 1.0 / np.sqrt(fi)
            self.p[f"W{k}"] = torch.from_numpy(r.uniform(-lim, lim, size=(fi, fo)).astype(np.float32)).cuda()
            self.p[f"b{k}"] = torch.zeros(fo, dtype=torch.float32, device="cuda")
        self.m = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.v = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.g = {k: torch.zeros_like(v) for k, v in self.p.items()}
        self.t = 0
        # input normalisation (set from the training set)
        self.mu = torch.zeros(n_in, dtype=torch.float32, device="cuda")
        self.sd = torch.ones(n_in, dtype=torch.float32, device="cuda")

    def _norm(self, X):
        import torch
        X = X.contiguous()
        Xn = torch.empty_like(X)
        nb.check(nb.lib().negf_mlp_normalize(X.shape[0], self.F, nb._ptr(X), nb._ptr(self.mu), nb._ptr(self.sd),
                                             nb._ptr(Xn), nb._stream()), "negf_mlp_normalize")
        return Xn

    def set_normalisation(self, X):
        """Input standardisation from the training set (column means and standard deviations)."""
        import torch
        X = X.contiguous()
        scratch = torch.empty(65 * self.F, dtype=torch.float64, device="cuda")
        nb.check(nb.lib().negf_mlp_moments(X.shape[0], self.F, nb._ptr(X), nb._ptr(self.mu), nb._ptr(self.sd),
                                           nb._ptr(scratch), nb._stream()), "negf_mlp_moments")

    def loss(self, Y, T):
        """Mean squared error of a batch (the training objective), in the library's kernel."""
        import torch
        out = torch.empty(1, dtype=torch.float64, device="cuda")
        scratch = torch.empty(64, dtype=torch.float64, device="cuda")
        nb.check(nb.lib().negf_mlp_mse(Y.numel(), nb._ptr(Y.contiguous()), nb._ptr(T.contiguous()), nb._ptr(out),
                                       nb._ptr(scratch), nb._stream()), "negf_mlp_mse")
        return out

    def state(self):
        """Checkpoint of the training state: parameters, Adam moments, step count and
        input standardisation, as host float32 arrays."""
        d = {"t": np.array([self.t], dtype=np.int64), "mu": self.mu.cpu().numpy(), "sd": self.sd.cpu().numpy()}
        for k in self.p:
            d[f"p_{k}"] = self.p[k].cpu().numpy()
            d[f"m_{k}"] = self.m[k].cpu().numpy()
            d[f"v_{k}"] = self.v[k].cpu().numpy()
        return d

    def save(self, path):
        """Write the checkpoint (safetensors: plain arrays, nothing executable)."""
        from safetensors.numpy import save_file
        save_file({k: np.ascontiguousarray(v) for k, v in self.state().items()}, path)

    def load(self, path):
        """Restore a checkpoint written by save() (shapes must match this network)."""
        import torch
        from safetensors.numpy import load_file
        d = load_file(path)
        for k in self.p:
            for pre, tgt in (("p", self.p), ("m", self.m), ("v", self.v)):
                a = d[f"{pre}_{k}"]
                if tuple(a.shape) != tuple(tgt[k].shape):
                    raise ValueError(f"checkpoint {pre}_{k} has shape {a.shape}, the network {tuple(tgt[k].shape)}")
                tgt[k].copy_(torch.from_numpy(a))
        self.mu.copy_(torch.from_numpy(d["mu"]))
        self.sd.copy_(torch.from_numpy(d["sd"]))
        self.t = int(d["t"][0])

    def forward(self, X):
        import torch
        L = nb.lib()
        n = X.shape[0]
        Xn = self._norm(X)
        A1 = torch.empty(n, self.H, dtype=torch.float32, device="cuda")
        A2 = torch.empty_like(A1)
        Y = torch.empty(n, self.O, dtype=torch.float32, device="cuda")
        p = self.p
        nb.check(L.negf_mlp_forward(n, self.F, self.H, self.O, nb._ptr(Xn), nb._ptr(p["W1"]), nb._ptr(p["b1"]),
                                    nb._ptr(p["W2"]), nb._ptr(p["b2"]), nb._ptr(p["W3"]), nb._ptr(p["b3"]),
                                    nb._ptr(A1), nb._ptr(A2), nb._ptr(Y), nb._stream()), "negf_mlp_forward")
        return Y, (Xn, A1, A2)

    def backward(self, cache, Y, T):
        import torch
        L = nb.lib()
        Xn, A1, A2 = cache
        n = Xn.shape[0]
        dY = torch.empty_like(Y)
        dZ2 = torch.empty_like(A2)
        dZ1 = torch.empty_like(A1)
        p, g = self.p, self.g
        nb.check(L.negf_mlp_backward(n, self.F, self.H, self.O, nb._ptr(Xn), nb._ptr(p["W2"]), nb._ptr(p["W3"]),
                                     nb._ptr(A1), nb._ptr(A2), nb._ptr(Y), nb._ptr(T), nb._ptr(g["W1"]),
                                     nb._ptr(g["b1"]), nb._ptr(g["W2"]), nb._ptr(g["b2"]), nb._ptr(g["W3"]),
                                     nb._ptr(g["b3"]), nb._ptr(dY), nb._ptr(dZ2), nb._ptr(dZ1), nb._stream()),
                 "negf_mlp_backward")
        return g

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        L = nb.lib()
        self.t += 1
        for k in self.p:
            nb.check(L.negf_mlp_adam_step(self.p[k].numel(), nb._ptr(self.p[k]), nb._ptr(self.g[k]),
                                          nb._ptr(self.m[k]), nb._ptr(self.v[k]), self.t, C.c_float(lr),
                                          C.c_float(beta1), C.c_float(beta2), C.c_float(eps), nb._stream()),
                     "negf_mlp_adam_step")

    def infer_bf16(self, X):
        import torch
        L = nb.lib()
        n = X.shape[0]
        Xn = self._norm(X)

        def bf(t):
            o = torch.empty(t.numel(), dtype=torch.int16, device="cuda")
            nb.check(L.negf_mlp_to_bf16(nb._ptr(t), nb._ptr(o), t.numel(), nb._stream()), "negf_mlp_to_bf16")
            return o

        Xb, W1b, W2b, W3b = bf(Xn), bf(self.p["W1"]), bf(self.p["W2"]), bf(self.p["W3"])
        scratch = torch.empty(2 * n * self.H, dtype=torch.int16, device="cuda")
        Y = torch.empty(n, self.O, dtype=torch.float32, device="cuda")
        nb.check(L.negf_mlp_infer_bf16(n, self.F, self.H, self.O, nb._ptr(Xb), nb._ptr(W1b), nb._ptr(self.p["b1"]),
                                       nb._ptr(W2b), nb._ptr(self.p["b2"]), nb._ptr(W3b), nb._ptr(self.p["b3"]),
                                       nb._ptr(scratch), nb._ptr(Y), nb._stream()), "negf_mlp_infer_bf16")
        return Y

    def train(self, X, T, epochs=5, batch=65536, lr=1e-3, seed=0, log=None, normalise=True):
        import torch
        if normalise:
            self.set_normalisation(X)
        n = X.shape[0]
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        losses = []
        for ep in range(epochs):
            perm = torch.randperm(n, device="cuda", generator=g)
            tot = 0.0
            for s in range(0, n, batch):
                idx = perm[s:s + batch]
                Xb, Tb = X[idx].contiguous(), T[idx].contiguous()
                Y, cache = self.forward(Xb)
                self.backward(cache, Y, Tb)
                self.adam(lr)
                tot += float(self.loss(Y, Tb).item()) * idx.numel()
            losses.append(tot / n)
            if log:
                log(f"epoch {ep + 1}/{epochs} mse {losses[-1]:.4e}")
        return losses


def solve_leads(problems: List[nb.Problem], side: int, seed=None, opts=None):
    """Decimation for every point (optionally seeded); returns the binding's dict."""
    return nb.obc_surface(problems, side, opts=opts, seed=seed)
