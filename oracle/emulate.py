"""Diagnostic emulation of the single-precision-product variants of RGF.

Not a reference for parity (the FP64 sweeps in ``rgf`` are); this module
predicts, on the CPU, what error the variants with complex64 products reach,
so that the GPU variant can be judged against an expectation.

Products marked single are formed from operands rounded to complex64 with a
complex64 NumPy matmul (single-precision accumulation) and widened back;
inversions, block sums and residuals stay complex128.

Variants (``mode``):
  "fp64"      -- every product in complex128 (equals ``rgf``)
  "fp32"      -- every sweep product single, no refinement
  "refine"    -- backward retarded products single, each block followed by
                 one double-precision residual correction through g_i; every
                 other product double:
                   retarded  (local identities of the backward step)
                     r_lo = -G_{i+1,i+1} A_{i+1,i} - G_{i+1,i} M_i ;  G_{i+1,i} += r_lo g_i
                     r_d  = I - M_i G_ii - A_{i,i+1} G_{i+1,i}     ;  G_ii     += g_i r_d
                     r_up = -A_{i,i+1} G_{i+1,i+1} - M_i G_{i,i+1} ;  G_{i,i+1} += g_i r_up
                 both lesser sweeps stay in double: each of the five backward
                 products alone leaves ~1e-5 in G^< when single, and single
                 forward products with one residual correction
                 (r = B_i - M_i g^<_i M_i^H, g^<_i += g_i r g_i^H) still leave
                 ~3e-7 in g^<, which the backward sweep amplifies to ~7e-6 on a
                 60-block device.  ``lesser(..., mode="refine1")`` keeps that
                 variant for the record.
"""
from __future__ import annotations

import numpy as np

inv = np.linalg.inv


def mm32(a, b):
    return (a.astype(np.complex64) @ b.astype(np.complex64)).astype(np.complex128)


def mm64(a, b):
    return a @ b


def retarded(Ad, Au, Al, mode="refine"):
    nb = len(Ad)
    fw = mm32 if mode == "fp32" else mm64
    bw = mm64 if mode == "fp64" else mm32
    g = [None] * nb
    M = [None] * nb
    X = [None] * (nb - 1)
    M[0] = Ad[0]
    g[0] = inv(M[0])
    for i in range(1, nb):
        X[i - 1] = fw(g[i - 1], Au[i - 1])
        M[i] = Ad[i] - fw(Al[i - 1], X[i - 1])
        g[i] = inv(M[i])
    Gd = [None] * nb
    Gu = [None] * (nb - 1)
    Gl = [None] * (nb - 1)
    Gd[nb - 1] = g[nb - 1]
    eye = np.eye(Ad[0].shape[0])
    for i in range(nb - 2, -1, -1):
        W = bw(Al[i], g[i])
        Gl[i] = -bw(Gd[i + 1], W)
        Gu[i] = -bw(X[i], Gd[i + 1])
        Gd[i] = g[i] - bw(X[i], Gl[i])
        if mode == "refine":
            r_lo = -(Gd[i + 1] @ Al[i]) - Gl[i] @ M[i]
            Gl[i] = Gl[i] + mm32(r_lo, g[i])
            r_d = eye - M[i] @ Gd[i] - Au[i] @ Gl[i]
            Gd[i] = Gd[i] + mm32(g[i], r_d)
            r_up = -(Au[i] @ Gd[i + 1]) - M[i] @ Gu[i]
            Gu[i] = Gu[i] + mm32(g[i], r_up)
    return dict(g=g, M=M, X=X, Gd=Gd, Gu=Gu, Gl=Gl)


def lesser(R, Au, Al, sig_diag, mode="refine"):
    g, M, X, Gd, Gu = R["g"], R["M"], R["X"], R["Gd"], R["Gu"]
    nb = len(g)
    mm = mm32 if mode in ("fp32", "refine1") else mm64
    gl = [None] * nb
    B = [None] * nb
    B[0] = sig_diag[0]
    gl[0] = mm(mm(g[0], B[0]), g[0].conj().T)
    if mode == "refine1":
        r = B[0] - M[0] @ gl[0] @ M[0].conj().T
        gl[0] = gl[0] + mm32(mm32(g[0], r), g[0].conj().T)
    for i in range(1, nb):
        # with a residual correction B_i is formed in double: the residual needs it
        mb = mm64 if mode == "refine1" else mm
        B[i] = sig_diag[i] + mb(mb(Al[i - 1], gl[i - 1]), Al[i - 1].conj().T)
        gl[i] = mm(mm(g[i], B[i]), g[i].conj().T)
        if mode == "refine1":
            r = B[i] - M[i] @ gl[i] @ M[i].conj().T
            gl[i] = gl[i] + mm32(mm32(g[i], r), g[i].conj().T)
    if mode in ("refine", "refine1"):
        mm = mm64
    Ld = [None] * nb
    Lu = [None] * (nb - 1)
    Ld[nb - 1] = gl[nb - 1]
    for i in range(nb - 2, -1, -1):
        V = mm(Al[i], gl[i])
        Q = -mm(Gu[i], V)
        Z = mm(X[i], Ld[i + 1])
        Ld[i] = gl[i] + mm(Z, X[i].conj().T) + Q - Q.conj().T
        Lu[i] = mm(V.conj().T, Gd[i + 1].conj().T) - Z
    return dict(gl=gl, Ld=Ld, Lu=Lu)
