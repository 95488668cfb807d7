"""Brute-force dense solution of Eq. (1) and Eq. (2) -- the definition.

G^R = A^{-1} with A = E S - H - Sigma^R (Eq. (1), C^R = (A - B^R)^{-1}),
G^< = G^R Sigma^< G^R^H and G^> = G^R Sigma^> G^R^H (Eq. (2) solved for C^<>).
The matrix is assembled in full (N = nb * b) and inverted with LAPACK; only
small systems (N up to a few thousand) are meant to go through here.

Also holds the explicit finite-lead construction that pins the orientation of
the lead self-energies without using the decimation.
"""
from __future__ import annotations

import numpy as np

from . import leads as _leads


def assemble_full(dev, E: float, sig_left=None, sig_right=None, with_scattering=True) -> np.ndarray:
    """Full A = E S - H - Sigma^R_scatt - Sigma^R_L (block 0) - Sigma^R_R (block nb-1)."""
    nb, b = dev.nb, dev.b
    N = nb * b
    A = np.zeros((N, N), dtype=np.complex128)
    for i in range(nb):
        sl = slice(i * b, (i + 1) * b)
        A[sl, sl] = E * dev.s_diag(i) - dev.H_diag[i]
        if with_scattering and dev.sig_r is not None:
            A[sl, sl] -= dev.sig_r[i]
    for i in range(nb - 1):
        s0 = slice(i * b, (i + 1) * b)
        s1 = slice((i + 1) * b, (i + 2) * b)
        up = E * dev.s_upper(i) - dev.H_upper[i]
        A[s0, s1] = up
        A[s1, s0] = up.conj().T
    if sig_left is not None:
        A[:b, :b] -= sig_left
    if sig_right is not None:
        A[N - b:, N - b:] -= sig_right
    return A


def block_diag_sigma(dev, lead_l, lead_r, with_scattering=True) -> np.ndarray:
    """Full block-diagonal self-energy with the given lead blocks at the ends."""
    nb, b = dev.nb, dev.b
    N = nb * b
    S = np.zeros((N, N), dtype=np.complex128)
    S[:b, :b] += lead_l
    S[N - b:, N - b:] += lead_r
    return S


def solve_point(dev, E, eta, mu_l=0.0, mu_r=0.0, kT=0.025, tol=_leads.TAU_DEFAULT, max_iter=100):
    """Dense G^R, G^<, G^> and T at one energy (leads by decimation)."""
    nb, b = dev.nb, dev.b
    N = nb * b
    L = _leads.lead_self_energy(dev, 0, E, eta, tol, max_iter)
    R = _leads.lead_self_energy(dev, 1, E, eta, tol, max_iter)
    A = assemble_full(dev, E, L.sigma_r, R.sigma_r)
    G = np.linalg.inv(A)
    fl = _leads.fermi(E - mu_l, kT)
    fr = _leads.fermi(E - mu_r, kT)
    sl_l, sg_l = _leads.lesser_greater(L.gamma, fl)
    sl_r, sg_r = _leads.lesser_greater(R.gamma, fr)
    Sl = block_diag_sigma(dev, sl_l, sl_r)
    Sg = block_diag_sigma(dev, sg_l, sg_r)
    if dev.sig_l is not None:
        for i in range(nb):
            sl = slice(i * b, (i + 1) * b)
            Sl[sl, sl] += dev.sig_l[i]
            Sg[sl, sl] += dev.sig_g[i]
    GH = G.conj().T
    Gl = G @ Sl @ GH
    Gg = G @ Sg @ GH
    G1N = G[:b, N - b:]
    GN1 = G[N - b:, :b]
    T_lr = float(np.real(np.trace(L.gamma @ G1N @ R.gamma @ G1N.conj().T)))
    T_rl = float(np.real(np.trace(R.gamma @ GN1 @ L.gamma @ GN1.conj().T)))
    return dict(G=G, Gl=Gl, Gg=Gg, T=T_rl, T_lr=T_lr, T_rl=T_rl, A=A, lead_l=L, lead_r=R, fl=fl, fr=fr)


def blocks_of(M: np.ndarray, nb: int, b: int):
    """(diag [nb,b,b], upper [nb-1,b,b], lower [nb-1,b,b]) blocks of a full matrix."""
    d = np.stack([M[i * b:(i + 1) * b, i * b:(i + 1) * b] for i in range(nb)])
    u = np.stack([M[i * b:(i + 1) * b, (i + 1) * b:(i + 2) * b] for i in range(nb - 1)]) if nb > 1 else np.zeros((0, b, b), M.dtype)
    lo = np.stack([M[(i + 1) * b:(i + 2) * b, i * b:(i + 1) * b] for i in range(nb - 1)]) if nb > 1 else np.zeros((0, b, b), M.dtype)
    return d, u, lo


def explicit_lead_self_energy(dev, side: int, E: float, eta: float, n_cells: int = 400) -> np.ndarray:
    """Lead self-energy from an explicit finite lead of ``n_cells`` cells.

    The lead is written out cell by cell from the raw device blocks as it
    sits in the physical structure: to the left of block 0 the cells repeat
    (H_00, S_00) joined by (H_01, S_01); to the right of block nb-1 they
    repeat (H_{N-1,N-1}, S_{N-1,N-1}) joined by the last coupling.  The lead
    matrix z S - H is inverted densely and the block next to the device
    gives Sigma = (zS - H)_{dev,lead} g_lead (zS - H)_{lead,dev}.  With
    eta > 0 the far end is screened after ~v/eta cells, so this converges to
    the semi-infinite result without any recursion.
    """
    b, nb = dev.b, dev.nb
    z = complex(E, eta)
    if side == 0:
        h0, s0 = dev.H_diag[0], dev.s_diag(0)
        h01, s01 = dev.H_upper[0], dev.s_upper(0)   # cell j -> cell j+1 (towards the device)
    else:
        h0, s0 = dev.H_diag[nb - 1], dev.s_diag(nb - 1)
        h01, s01 = dev.H_upper[nb - 2], dev.s_upper(nb - 2)
    n = n_cells
    M = np.zeros((n * b, n * b), dtype=np.complex128)
    for j in range(n):
        sj = slice(j * b, (j + 1) * b)
        M[sj, sj] = z * s0 - h0
    for j in range(n - 1):
        s_a = slice(j * b, (j + 1) * b)
        s_b = slice((j + 1) * b, (j + 2) * b)
        up = z * s01 - h01              # (zS - H) from cell j to cell j+1 (left to right)
        lo = z * s01.conj().T - h01.conj().T
        M[s_a, s_b] = up
        M[s_b, s_a] = lo
    Minv = np.linalg.inv(M)
    if side == 0:
        # lead cells ordered left to right; the last one touches device block 0
        g = Minv[(n - 1) * b:, (n - 1) * b:]
        c_dev_lead = z * s01.conj().T - h01.conj().T      # (zS-H)_{0,-1}
        c_lead_dev = z * s01 - h01                        # (zS-H)_{-1,0}
    else:
        # lead cells ordered left to right; the first one touches block nb-1
        g = Minv[:b, :b]
        c_dev_lead = z * s01 - h01                        # (zS-H)_{N-1,N}
        c_lead_dev = z * s01.conj().T - h01.conj().T
    return c_dev_lead @ g @ c_lead_dev
