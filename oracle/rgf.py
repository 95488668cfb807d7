"""Recursive Green's function (RGF) selected inversion -- FP64 oracle.

The paper names RGF as the sequential solver for Eq. (1) and Eq. (2) on the
block-tridiagonal (BT) operators and asks only for the entries of C inside the
sparsity pattern of A and B (Section II, the paragraphs after Fig. 3).  The
recursions below are the textbook forward/backward Schur-complement sweeps
(Svizhenko et al., J. Appl. Phys. 91, 2343 (2002), cited by the paper for
RGF), written out in the order the sweeps run.

Blocks are numbered 0..nb-1.  Inputs are the A blocks:
  A_ii      = E S_ii - H_ii - Sigma^R_sc,ii - [i=0] Sigma^R_L - [i=nb-1] Sigma^R_R
  A_{i,i+1} = E S_{i,i+1} - H_{i,i+1},   A_{i+1,i} = A_{i,i+1}^H   (E real)

Retarded, forward:  g_0 = A_00^{-1};  X_{i-1} = g_{i-1} A_{i-1,i};
                    g_i = (A_ii - A_{i,i-1} X_{i-1})^{-1}
Retarded, backward: G_{N-1,N-1} = g_{N-1};  for i = N-2 .. 0:
                    G_{i+1,i} = -G_{i+1,i+1} A_{i+1,i} g_i
                    G_{i,i+1} = -X_i G_{i+1,i+1}
                    G_ii      =  g_i - X_i G_{i+1,i}
Lesser/greater (Sigma block diagonal), forward:
                    g^<_0 = g_0 Sigma^<_00 g_0^H
                    g^<_i = g_i (Sigma^<_ii + A_{i,i-1} g^<_{i-1} A_{i,i-1}^H) g_i^H
Lesser/greater, backward: G^<_{N-1,N-1} = g^<_{N-1};  for i = N-2 .. 0:
                    V = A_{i+1,i} g^<_i;  Q = -G_{i,i+1} V;  Z = X_i G^<_{i+1,i+1}
                    G^<_ii      = g^<_i + Z X_i^H + Q - Q^H
                    G^<_{i,i+1} = V^H G_{i+1,i+1}^H - Z
                    G^<_{i+1,i} = -(G^<_{i,i+1})^H
  (the same formulas with Sigma^> give G^>; they use that Sigma^<> is
  anti-Hermitian so that g^<> is too).
Transmission: C_0 = g_0; C_i = -g_i A_{i,i-1} C_{i-1}; G_{N-1,0} = C_{N-1};
              T = Tr[Gamma_R G_{N-1,0} Gamma_L G_{N-1,0}^H].
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import leads as _leads

inv = np.linalg.inv


def assemble_blocks(dev, E: float, sig_left=None, sig_right=None, with_scattering=True):
    """A-blocks (diag [nb], upper [nb-1], lower [nb-1]) at real energy E."""
    nb = dev.nb
    Ad = []
    for i in range(nb):
        a = E * dev.s_diag(i) - dev.H_diag[i]
        if with_scattering and dev.sig_r is not None:
            a = a - dev.sig_r[i]
        if i == 0 and sig_left is not None:
            a = a - sig_left
        if i == nb - 1 and sig_right is not None:
            a = a - sig_right
        Ad.append(a)
    Au = [E * dev.s_upper(i) - dev.H_upper[i] for i in range(nb - 1)]
    Al = [u.conj().T for u in Au]
    return Ad, Au, Al


def retarded(Ad, Au, Al):
    """Forward and backward retarded sweeps.  Returns (g, X, Gd, Gu, Gl)."""
    nb = len(Ad)
    g = [None] * nb
    X = [None] * max(nb - 1, 0)
    g[0] = inv(Ad[0])
    for i in range(1, nb):
        X[i - 1] = g[i - 1] @ Au[i - 1]
        g[i] = inv(Ad[i] - Al[i - 1] @ X[i - 1])
    Gd = [None] * nb
    Gu = [None] * max(nb - 1, 0)
    Gl = [None] * max(nb - 1, 0)
    Gd[nb - 1] = g[nb - 1]
    for i in range(nb - 2, -1, -1):
        Gl[i] = -Gd[i + 1] @ Al[i] @ g[i]
        Gu[i] = -X[i] @ Gd[i + 1]
        Gd[i] = g[i] - X[i] @ Gl[i]
    return g, X, Gd, Gu, Gl


def lesser(g, X, Gd, Gu, Al, sig_diag):
    """Forward and backward sweeps for G^< (or G^> with Sigma^>).

    ``sig_diag[i]`` is the full block-diagonal Sigma^<_ii (leads + scattering).
    Returns (g^<, G^<_diag, G^<_upper).
    """
    nb = len(g)
    gl = [None] * nb
    gl[0] = g[0] @ sig_diag[0] @ g[0].conj().T
    for i in range(1, nb):
        Bt = sig_diag[i] + Al[i - 1] @ gl[i - 1] @ Al[i - 1].conj().T
        gl[i] = g[i] @ Bt @ g[i].conj().T
    Ld = [None] * nb
    Lu = [None] * max(nb - 1, 0)
    Ld[nb - 1] = gl[nb - 1]
    for i in range(nb - 2, -1, -1):
        V = Al[i] @ gl[i]
        Q = -Gu[i] @ V
        Z = X[i] @ Ld[i + 1]
        Ld[i] = gl[i] + Z @ X[i].conj().T + Q - Q.conj().T
        Lu[i] = V.conj().T @ Gd[i + 1].conj().T - Z
    return gl, Ld, Lu


def corner_block(g, Al):
    """G_{N-1,0} from the left-connected recursion C_i = -g_i A_{i,i-1} C_{i-1}."""
    C = g[0]
    for i in range(1, len(g)):
        C = -g[i] @ Al[i - 1] @ C
    return C


def transmission(g, Al, gamma_l, gamma_r) -> float:
    C = corner_block(g, Al)
    return float(np.real(np.trace(gamma_r @ C @ gamma_l @ C.conj().T)))


@dataclasses.dataclass
class PointResult:
    E: float
    GR_diag: np.ndarray
    GR_upper: np.ndarray
    GR_lower: np.ndarray
    GL_diag: Optional[np.ndarray] = None
    GL_upper: Optional[np.ndarray] = None
    GG_diag: Optional[np.ndarray] = None
    GG_upper: Optional[np.ndarray] = None
    T: Optional[float] = None
    lead_l: object = None
    lead_r: object = None
    fl: float = 0.0
    fr: float = 0.0


def _stack(blocks, b):
    if len(blocks) == 0:
        return np.zeros((0, b, b), dtype=np.complex128)
    return np.stack(blocks)


def solve_point(dev, E, eta, mu_l=0.0, mu_r=0.0, kT=0.025, lesser_greater=True,
                greater=False, want_T=False, tol=_leads.TAU_DEFAULT, max_iter=100) -> PointResult:
    """One (E, k) point: both leads, G^R, optionally G^< (and G^>), optionally T."""
    b, nb = dev.b, dev.nb
    L = _leads.lead_self_energy(dev, 0, E, eta, tol, max_iter)
    R = _leads.lead_self_energy(dev, 1, E, eta, tol, max_iter)
    Ad, Au, Al = assemble_blocks(dev, E, L.sigma_r, R.sigma_r)
    g, X, Gd, Gu, Gl = retarded(Ad, Au, Al)
    res = PointResult(E, _stack(Gd, b), _stack(Gu, b), _stack(Gl, b), lead_l=L, lead_r=R)
    res.fl = _leads.fermi(E - mu_l, kT)
    res.fr = _leads.fermi(E - mu_r, kT)
    if lesser_greater:
        kinds = [0, 1] if greater else [0]
        for kind in kinds:
            lead_l = _leads.lesser_greater(L.gamma, res.fl)[kind]
            lead_r = _leads.lesser_greater(R.gamma, res.fr)[kind]
            sig = []
            for i in range(nb):
                s = np.zeros((b, b), dtype=np.complex128)
                if dev.sig_l is not None:
                    s = s + (dev.sig_l[i] if kind == 0 else dev.sig_g[i])
                if i == 0:
                    s = s + lead_l
                if i == nb - 1:
                    s = s + lead_r
                sig.append(s)
            _, Ld, Lu = lesser(g, X, Gd, Gu, Al, sig)
            if kind == 0:
                res.GL_diag, res.GL_upper = _stack(Ld, b), _stack(Lu, b)
            else:
                res.GG_diag, res.GG_upper = _stack(Ld, b), _stack(Lu, b)
    if want_T:
        res.T = transmission(g, Al, L.gamma, R.gamma)
    return res
