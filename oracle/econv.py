"""Energy convolution of Eq. (3) on a uniform grid -- FP64 oracle (TEST
INFRASTRUCTURE ONLY).

Eq. (3) builds a self-energy from two Green's-function-like quantities by an
integral over energy, B(E) ~ int dE' (M1 C1(E - E') M2) (.) C2(E'), with (.)
an element-wise product; the paper evaluates it with FFTs in the time domain
(Section II, the paragraph after Fig. 3).  With M1 = M2 = I and the
element-wise product (the GW form Sigma_ij(E) ~ int dE' G_ij(E - E') W_ij(E')),
on a uniform grid E_e = E_0 + e dE (e = 0..n_e-1) for C1 = G and frequencies
w_k = (k - k0) dE (k = 0..n_w-1) for C2 = W, the integral becomes the
discrete convolution

    B[e][x] = scale * sum_{k=0}^{n_w-1} G[e + k0 - k][x] * W[k][x]

for every element x (a matrix entry (i, j) of the selected blocks), with G
taken as zero outside the grid, and scale carrying dE and the physical
prefactor (e.g. i dE / 2pi).  This is the definition, written out as the sum
over k: no FFT, no reordering.  Arrays are energy-major: G [n_e][n_el],
W [n_w][n_el], B [n_e][n_el], complex128.
"""
from __future__ import annotations

import numpy as np


def energy_convolution(G: np.ndarray, W: np.ndarray, k0: int, scale: complex = 1.0) -> np.ndarray:
    """B[e] = scale * sum_k G[e + k0 - k] W[k] (element-wise over the trailing axis)."""
    G = np.asarray(G, dtype=np.complex128)
    W = np.asarray(W, dtype=np.complex128)
    n_e, n_w = G.shape[0], W.shape[0]
    B = np.zeros_like(G)
    for k in range(n_w):
        shift = k0 - k                      # B[e] += G[e + shift] W[k]
        lo = max(0, -shift)
        hi = min(n_e, n_e - shift)
        if lo < hi:
            B[lo:hi] += G[lo + shift:hi + shift] * W[k]
    return scale * B


def to_element_major(X: np.ndarray) -> np.ndarray:
    """(E; i,j) -> (i,j; E): the layout change between the linear solves (all
    entries of a few energies) and the convolution (a few entries at all
    energies), Fig. 2."""
    return np.ascontiguousarray(np.swapaxes(X, 0, 1))
