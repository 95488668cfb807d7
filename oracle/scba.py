"""Self-consistent Born loop around Eq. (1)-(3) -- FP64 oracle (TEST
INFRASTRUCTURE ONLY).

Fig. 1 alternates two steps until they agree: the electron Green's functions
G^{R,<,>} are solved from Eq. (1) and Eq. (2) with the scattering
self-energies Sigma^{R,<,>}, and the self-energies are rebuilt from G^<> by
the energy convolution of Eq. (3).  Here the second propagator of Eq. (3) is
a fixed boson bath W^<> (its own loop through the polarisation, the bosonic
half of Fig. 1, is not run), M1 = M2 = I, and the product is element-wise
over the diagonal blocks, the self-energies being block diagonal as the
sweeps require.  On a uniform grid E_e = E_0 + e dE, with W sampled at
w_k = (k - k0) dE:

    F^<>_ii(E_e) = scale * sum_k G^<>_ii(E_e - w_k) (.) W^<>[k]

(the plain sum of ``econv``; G is zero outside the grid), and the retarded
self-energy is the anti-Hermitian combination (F^> - F^<) / 2 (the
Hermitian, principal-value part is not formed).  With several transverse
momenta k (one device H(k) each, Eq. (1)-(3) omit k) the self-energies are
taken independent of k and G^<> in the convolution is the average over the
k-points of each energy (the local-in-k reading).

Iteration n (n = 0, 1, ...) solves every energy with Sigma_n, forms F from the
new G^<>, and measures

    r_n = sqrt(sum ||F^< - Sigma^<_n||_F^2 + ||F^> - Sigma^>_n||_F^2)
          / sqrt(sum ||F^<||_F^2 + ||F^>||_F^2)

over all energies and blocks (0 when both norms are 0).  It stops when
r_n <= tol, or at n = max_iter - 1, and returns Sigma_n with the Green's
functions that Sigma_n produced (so G^<> = G Sigma^<>_n G^H holds for the
returned pair); otherwise Sigma_{n+1} = Sigma_n + m (F - Sigma_n) for both
kinds, and Sigma^R_{n+1} = (Sigma^>_{n+1} - Sigma^<_{n+1}) / 2.

With a memory M > 0 the update is Anderson's (Pulay's) extrapolation instead:
x = (Sigma^<, Sigma^>), f = F - x, and the differences dx_j, df_j of the last
k = min(n, M) pairs (x, f);  gamma minimises ||f_n - sum_j gamma_j df_j||
(the normal equations A gamma = r with A_ij = Re <df_i, df_j>,
r_i = Re <df_i, f_n>, A's diagonal raised by 1e-12 trace(A) / k), and
x_{n+1} = x_n + m f_n - sum_j gamma_j (dx_j + m df_j)  (D. G. Anderson,
J. ACM 12, 547 (1965); P. Pulay, Chem. Phys. Lett. 73, 393 (1980)).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np

from . import econv as _econv
from . import rgf as _rgf


def retarded_from(sig_l: np.ndarray, sig_g: np.ndarray) -> np.ndarray:
    """Sigma^R = (Sigma^> - Sigma^<) / 2: the anti-Hermitian part that Sigma^R - Sigma^A = Sigma^> - Sigma^<
    fixes."""
    return 0.5 * (sig_g - sig_l)


def residual(Fl, Fg, Sl, Sg) -> float:
    num = float(np.sum(np.abs(Fl - Sl) ** 2) + np.sum(np.abs(Fg - Sg) ** 2))
    den = float(np.sum(np.abs(Fl) ** 2) + np.sum(np.abs(Fg) ** 2))
    if den == 0.0:
        return 0.0 if num == 0.0 else math.inf
    return math.sqrt(num / den)


@dataclasses.dataclass
class ScbaResult:
    sig_r: np.ndarray          # [n_e][nb][b][b]
    sig_l: np.ndarray
    sig_g: np.ndarray
    points: List[_rgf.PointResult]
    n_iter: int                # solves performed
    history: List[float]       # r_0 .. r_{n_iter - 1}
    converged: bool


def solve_all(dev, energies, eta, mu_l, mu_r, kT, sig_r, sig_l, sig_g):
    """Eq. (1) and (2) at every energy with that energy's scattering self-energies."""
    pts = []
    for e, E in enumerate(energies):
        de = dataclasses.replace(dev, sig_r=sig_r[e], sig_l=sig_l[e], sig_g=sig_g[e])
        pts.append(_rgf.solve_point(de, float(E), eta, mu_l, mu_r, kT, lesser_greater=True, greater=True))
    return pts


def convolve(points, W_l, W_g, k0, scale):
    """F^<> of Eq. (3) from the diagonal blocks of every energy's G^<> (``points`` [e], or [k][e]
    for several k-points: the average over k)."""
    if isinstance(points[0], list):
        Gl = np.mean([np.stack([p.GL_diag for p in pk]) for pk in points], axis=0)
        Gg = np.mean([np.stack([p.GG_diag for p in pk]) for pk in points], axis=0)
    else:
        Gl = np.stack([p.GL_diag for p in points])
        Gg = np.stack([p.GG_diag for p in points])
    shp = Gl.shape
    n_w = W_l.shape[0]
    Fl = _econv.energy_convolution(Gl.reshape(shp[0], -1), W_l.reshape(n_w, -1), k0, scale)
    Fg = _econv.energy_convolution(Gg.reshape(shp[0], -1), W_g.reshape(n_w, -1), k0, scale)
    return Fl.reshape(shp), Fg.reshape(shp)


def anderson(x, f, dxs, dfs, mixing):
    """x_{n+1} from x_n, f_n and the differences of the previous pairs (lists, any order)."""
    k = len(dfs)
    if k == 0:
        return x + mixing * f
    DF = np.array(dfs)
    DX = np.array(dxs)
    A = np.real(DF.conj() @ DF.T)
    r = np.real(DF.conj() @ f)
    A = A + 1e-12 * np.trace(A) / k * np.eye(k)
    g = np.linalg.solve(A, r)
    return x + mixing * f - g @ (DX + mixing * DF)


def scba(dev, energies, eta, mu_l, mu_r, kT, W_l, W_g, k0, scale, mixing=0.5, tol=1e-10, max_iter=50,
         sig0=None, memory=0) -> ScbaResult:
    """The loop of Fig. 1 with a fixed bath.  ``sig0`` = (Sigma^<, Sigma^>) to start from
    (default zero: the ballistic solution is iteration 0); ``energies`` must be uniform, the
    spacing entering only through ``scale`` (i dE / 2 pi for the usual normalisation).  ``dev`` may
    be a list of devices (one per k-point, same block shape): the points are then [k][e]."""
    devs = dev if isinstance(dev, (list, tuple)) else None
    n_e, nb, b = len(energies), (devs or [dev])[0].nb, (devs or [dev])[0].b
    if sig0 is None:
        Sl = np.zeros((n_e, nb, b, b), dtype=np.complex128)
        Sg = np.zeros_like(Sl)
    else:
        Sl = np.array(sig0[0], dtype=np.complex128)
        Sg = np.array(sig0[1], dtype=np.complex128)
    Sr = retarded_from(Sl, Sg)
    hist = []
    prev, dxs, dfs = None, [], []
    for n in range(max_iter):
        if devs is None:
            pts = solve_all(dev, energies, eta, mu_l, mu_r, kT, Sr, Sl, Sg)
        else:
            pts = [solve_all(d, energies, eta, mu_l, mu_r, kT, Sr, Sl, Sg) for d in devs]
        Fl, Fg = convolve(pts, W_l, W_g, k0, scale)
        r = residual(Fl, Fg, Sl, Sg)
        hist.append(r)
        if r <= tol or n == max_iter - 1 or not math.isfinite(r):
            return ScbaResult(Sr, Sl, Sg, pts, n + 1, hist, r <= tol)
        if memory == 0:
            Sl = Sl + mixing * (Fl - Sl)
            Sg = Sg + mixing * (Fg - Sg)
        else:
            x = np.concatenate([Sl.ravel(), Sg.ravel()])
            f = np.concatenate([Fl.ravel(), Fg.ravel()]) - x
            if prev is not None:
                dxs.append(x - prev[0])
                dfs.append(f - prev[1])
                dxs, dfs = dxs[-memory:], dfs[-memory:]
            prev = (x, f)
            xn = anderson(x, f, dxs, dfs, mixing)
            h = xn.size // 2
            Sl = xn[:h].reshape(Sl.shape)
            Sg = xn[h:].reshape(Sg.shape)
        Sr = retarded_from(Sl, Sg)
    raise ValueError("max_iter must be at least 1")
