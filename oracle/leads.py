"""Open-boundary self-energies of the two semi-infinite leads.

The paper adds an open-boundary term to B^R in Eq. (1) without stating how
it is computed (Section II, the sentence after Eq. (3)).  This oracle uses
the Sancho-Rubio decimation (M. P. Lopez Sancho, J. M. Lopez Sancho,
J. Rubio, J. Phys. F 15, 851 (1985)) for the surface Green's function of a
lead that repeats the first (left) or last (right) device cell.

Conventions
-----------
z = E + i eta is used inside the lead only; the device itself stays at real
energy.  For a lead with cell (H0, S0) and coupling (H1, S1) from a cell to
the next cell *away from the device*:

    d     = z S0 - H0
    alpha = H1 - z S1          (surface cell -> next cell, minus sign of zS - H)
    beta  = H1^H - z S1^H      (next cell -> surface cell)

Left lead : H0 = H_00, S0 = S_00, H1 = H_01^H, S1 = S_01^H
Right lead: H0 = H_NN, S0 = S_NN, H1 = H_{N-1,N}, S1 = S_{N-1,N}

The surface Green's function solves g_s = (d - alpha g_s beta)^{-1}; the
retarded self-energy on the adjacent device block is Sigma^R = alpha g_s beta;
Gamma = i (Sigma^R - Sigma^R^H); Sigma^< = i f Gamma, Sigma^> = -i (1-f) Gamma.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TAU_DEFAULT = 1e-14


@dataclasses.dataclass
class LeadResult:
    g_surf: np.ndarray
    sigma_r: np.ndarray
    gamma: np.ndarray
    iters: int
    residual: float
    converged: bool


def fermi(x: float, kT: float) -> float:
    """Fermi-Dirac occupation 1 / (1 + exp(x / kT)), evaluated without overflow."""
    if kT <= 0.0:
        return 1.0 if x < 0 else (0.5 if x == 0 else 0.0)
    y = x / kT
    if y > 0:
        e = math.exp(-y)
        return e / (1.0 + e)
    return 1.0 / (1.0 + math.exp(y))


def lead_blocks(dev, side: int, E: float, eta: float):
    """(d, alpha, beta) of the left (side=0) or right (side=1) lead at z = E + i eta."""
    z = complex(E, eta)
    nb = dev.nb
    if side == 0:
        H0, S0 = dev.H_diag[0], dev.s_diag(0)
        H1, S1 = dev.H_upper[0].conj().T, dev.s_upper(0).conj().T
    else:
        H0, S0 = dev.H_diag[nb - 1], dev.s_diag(nb - 1)
        H1, S1 = dev.H_upper[nb - 2], dev.s_upper(nb - 2)
    d = z * S0 - H0
    alpha = H1 - z * S1
    beta = H1.conj().T - z * S1.conj().T
    return d, alpha, beta


def sancho_rubio(d, alpha, beta, tol=TAU_DEFAULT, max_iter=100):
    """Decimation for the surface Green's function.

    Start eps_s = eps = d, a = alpha, c = beta; each step, with g = eps^{-1}:
    eps_s -= a g c; eps -= a g c + c g a; a = a g a; c = c g c.  Stop when
    ||a||_F and ||c||_F both fall to tol * ||d||_F.  Returns
    (g_s = eps_s^{-1}, iterations, converged).
    """
    eps_s = d.copy()
    eps = d.copy()
    a = alpha.copy()
    c = beta.copy()
    dn = np.linalg.norm(d)
    it = 0
    converged = False
    for it in range(1, max_iter + 1):
        g = np.linalg.inv(eps)
        agc = a @ g @ c
        cga = c @ g @ a
        eps_s = eps_s - agc
        eps = eps - agc - cga
        a = a @ g @ a
        c = c @ g @ c
        if np.linalg.norm(a) <= tol * dn and np.linalg.norm(c) <= tol * dn:
            converged = True
            break
    return np.linalg.inv(eps_s), it, converged


def seeded_closure(eps, eps_s, a, c, d_seed):
    """Surface Green's function of the decimated chain closed with a seed.

    After k decimation steps the lead is the surface cell (eps_s) coupled by
    a, c to a cell whose onsite block, seen from the surface, is its own
    renormalisation from the decimated cells between them (eps - eps_s) plus
    the original onsite block and the exact self-energy of the undecimated
    lead beyond it: d - alpha g_s beta.  With g_s replaced by a seed g~
    (d_seed = d - alpha g~ beta):
        X = (eps - eps_s + d_seed)^{-1},  g = (eps_s - a X c)^{-1}.
    For g~ = g_s this is exact at every step; as a, c vanish it tends to
    eps_s^{-1}, the plain decimation result.
    """
    X = np.linalg.inv(eps - eps_s + d_seed)
    return np.linalg.inv(eps_s - a @ X @ c)


def seeded_sancho_rubio(d, alpha, beta, g_seed, accept=1e-8, tol=TAU_DEFAULT, max_iter=100):
    """Decimation seeded with a guess g~ of the surface Green's function.

    1. candidate g0 = (d - alpha g~ beta)^{-1}; accepted (0 steps) when its
       normalised Dyson residual is <= accept;
    2. otherwise plain decimation steps; after step k the seeded closure
       (seeded_closure) is accepted at the first k where its residual is
       <= accept;
    3. otherwise the plain result when the decimation converges.
    Returns (g_s, steps, how) with how in {"candidate", "closure", "plain"}.
    """
    d_seed = d - alpha @ g_seed @ beta
    g0 = np.linalg.inv(d_seed)
    if dyson_residual(d, alpha, beta, g0) <= accept:
        return g0, 0, "candidate"
    eps_s = d.copy()
    eps = d.copy()
    a = alpha.copy()
    c = beta.copy()
    dn = np.linalg.norm(d)
    it = 0
    for it in range(1, max_iter + 1):
        g = np.linalg.inv(eps)
        agc = a @ g @ c
        cga = c @ g @ a
        eps_s = eps_s - agc
        eps = eps - agc - cga
        a = a @ g @ a
        c = c @ g @ c
        gk = seeded_closure(eps, eps_s, a, c, d_seed)
        if dyson_residual(d, alpha, beta, gk) <= accept:
            return gk, it, "closure"
        if np.linalg.norm(a) <= tol * dn and np.linalg.norm(c) <= tol * dn:
            break
    return np.linalg.inv(eps_s), it, "plain"


def dyson_residual(d, alpha, beta, g_s) -> float:
    """r = ||(d - alpha g_s beta) g_s - I||_F / (||d - alpha g_s beta||_F ||g_s||_F)."""
    m = d - alpha @ g_s @ beta
    eye = np.eye(d.shape[0])
    return float(np.linalg.norm(m @ g_s - eye) / (np.linalg.norm(m) * np.linalg.norm(g_s)))


def lead_self_energy(dev, side: int, E: float, eta: float, tol=TAU_DEFAULT, max_iter=100) -> LeadResult:
    d, alpha, beta = lead_blocks(dev, side, E, eta)
    g_s, it, conv = sancho_rubio(d, alpha, beta, tol, max_iter)
    sig = alpha @ g_s @ beta
    gam = 1j * (sig - sig.conj().T)
    res = dyson_residual(d, alpha, beta, g_s)
    return LeadResult(g_s, sig, gam, it, res, conv)


def lesser_greater(gamma: np.ndarray, f: float):
    """Sigma^< = i f Gamma, Sigma^> = -i (1 - f) Gamma."""
    return 1j * f * gamma, -1j * (1.0 - f) * gamma
