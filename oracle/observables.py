"""Observables from the Green's function blocks (Section III: current, DOS).

The paper uses current conservation along the device as its validation of
the implementation (Section III, Fig. 5(b) inset) and shows the local density
of states (Fig. 5(a)).  Units: e = hbar = 1, one spin.
"""
from __future__ import annotations

import numpy as np


def interface_current(A_upper, GL_lower) -> float:
    """Spectral current through the interface between blocks i and i+1.

    j_i(E) = -2 Re Tr[A_{i,i+1} G^<_{i+1,i}]; with the Landauer convention of
    this package it equals (f_L - f_R) T(E) in the ballistic limit.
    """
    return float(-2.0 * np.real(np.trace(A_upper @ GL_lower)))


def currents(Au, GL_upper):
    """j_i for every interface from A_{i,i+1} and G^<_{i,i+1} (G^<_{i+1,i} = -G^<_{i,i+1}^H)."""
    return np.array([interface_current(Au[i], -GL_upper[i].conj().T) for i in range(len(Au))])


def lead_current(sig_l_lesser, sig_l_greater, GL_00, GG_00) -> float:
    """Current injected by the left lead: Tr[Sigma^<_L G^>_00 - Sigma^>_L G^<_00] (real part)."""
    return float(np.real(np.trace(sig_l_lesser @ GG_00 - sig_l_greater @ GL_00)))


def dos(GR_diag) -> np.ndarray:
    """Block-resolved density of states -Im Tr G_ii / pi."""
    return np.array([-np.imag(np.trace(g)) / np.pi for g in GR_diag])
