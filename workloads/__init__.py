"""Seeded synthetic inputs for the NEGF hot path.

This module only draws random numbers and lays out block-tridiagonal input
arrays.  It contains none of the method's arithmetic (no Green's functions,
no self-energies from leads, no inversions).  Both the CPU oracle and the GPU
path receive their inputs from here, so the two sides see identical data.

The paper solves Eq. (1)/(2) on block-tridiagonal operators obtained from a
DFT/MLWF Hamiltonian of a Si nano-ribbon (Section III, Fig. 4(a)).  Those
Hamiltonians are not available, so the generators below produce random
Hermitian block-tridiagonal operators with the same block shapes and a
comparable sparsity pattern.

Conventions
-----------
* Blocks are numbered 0..nb-1.  ``H_diag[i]`` is H_ii, ``H_upper[i]`` is
  H_{i,i+1}; the lower blocks are the Hermitian adjoints of the upper ones.
* ``S_diag``/``S_upper`` of ``None`` mean S = I.
* A complex Gaussian "N(0, s)" has Re and Im i.i.d. N(0, s^2/2), so that
  E|x|^2 = s^2.
* All arrays are C-contiguous complex128.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "BTDevice", "rng", "cgauss", "random_device", "chain_device",
    "folded_chain_device", "periodic_wire_device", "slab_device", "slab_lead",
    "slab_geometry", "scattering_self_energies", "k_device", "mixed_devices",
    "energy_grid", "DEVICE_MIX", "boson_bath",
]


def rng(seed: int) -> np.random.Generator:
    """PCG64 generator for ``seed``."""
    return np.random.Generator(np.random.PCG64(seed))


def cgauss(r: np.random.Generator, shape, std: float) -> np.ndarray:
    """Complex Gaussian with E|x|^2 = std^2 (Re, Im i.i.d. N(0, std^2/2))."""
    s = std / math.sqrt(2.0)
    return (r.standard_normal(shape) * s + 1j * (r.standard_normal(shape) * s)).astype(np.complex128)


@dataclasses.dataclass
class BTDevice:
    """A block-tridiagonal device description (all blocks b x b)."""
    H_diag: np.ndarray
    H_upper: np.ndarray
    S_diag: Optional[np.ndarray] = None
    S_upper: Optional[np.ndarray] = None
    sig_r: Optional[np.ndarray] = None   # retarded scattering self-energy, block diagonal
    sig_l: Optional[np.ndarray] = None   # lesser
    sig_g: Optional[np.ndarray] = None   # greater
    name: str = ""

    @property
    def nb(self) -> int:
        return int(self.H_diag.shape[0])

    @property
    def b(self) -> int:
        return int(self.H_diag.shape[1])

    def s_diag(self, i: int) -> np.ndarray:
        if self.S_diag is None:
            return np.eye(self.b, dtype=np.complex128)
        return self.S_diag[i]

    def s_upper(self, i: int) -> np.ndarray:
        if self.S_upper is None:
            return np.zeros((self.b, self.b), dtype=np.complex128)
        return self.S_upper[i]


def _herm(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(0.5 * (x + x.conj().T))


# --------------------------------------------------------------------------
# Small test systems
# --------------------------------------------------------------------------

def random_device(nb: int, b: int, seed: int, coupling_std: float = 0.3,
                  overlap: float = 0.0) -> BTDevice:
    """Dense random device of the small ballistic workload.

    On-site blocks: X with Re, Im ~ N(0, 1), H_ii = (X + X^H) / (2 sqrt(b));
    couplings: complex Gaussian with std ``coupling_std``; S = I unless
    ``overlap`` > 0, in which case S = I + a PSD perturbation of spectral
    norm <= ``overlap`` built as for the slab devices.
    """
    r = rng(seed)
    x = r.standard_normal((nb, b, b)) + 1j * r.standard_normal((nb, b, b))
    H_diag = (x + np.conj(np.transpose(x, (0, 2, 1)))) / (2.0 * math.sqrt(b))
    H_upper = cgauss(r, (nb - 1, b, b), coupling_std)
    dev = BTDevice(np.ascontiguousarray(H_diag), np.ascontiguousarray(H_upper), name=f"random{nb}x{b}")
    if overlap > 0.0:
        mask_d = np.ones((b, b), dtype=bool)
        mask_u = np.ones((b, b), dtype=bool)
        dev.S_diag, dev.S_upper = _overlap_from_pattern(r, nb, b, mask_d, mask_u, overlap)
    return dev


def chain_device(nb: int, eps: float = 0.0, t: float = 1.0) -> BTDevice:
    """1D tight-binding chain, one orbital per cell (b = 1), hopping -t."""
    H_diag = np.full((nb, 1, 1), eps, dtype=np.complex128)
    H_upper = np.full((nb - 1, 1, 1), -t, dtype=np.complex128)
    return BTDevice(H_diag, H_upper, name="chain")


def folded_chain_device(nb: int, b: int = 8, eps: float = 0.0, t: float = 1.0) -> BTDevice:
    """The 1D chain folded into cells of b sites (same physics as the chain)."""
    cell = np.zeros((b, b), dtype=np.complex128)
    for j in range(b):
        cell[j, j] = eps
    for j in range(b - 1):
        cell[j, j + 1] = -t
        cell[j + 1, j] = -t
    cpl = np.zeros((b, b), dtype=np.complex128)
    cpl[b - 1, 0] = -t
    H_diag = np.ascontiguousarray(np.broadcast_to(cell, (nb, b, b)))
    H_upper = np.ascontiguousarray(np.broadcast_to(cpl, (nb - 1, b, b)))
    return BTDevice(H_diag, H_upper, name="folded_chain")


def periodic_wire_device(nb: int, b: int, seed: int, coupling_std: float = 0.3) -> BTDevice:
    """A device whose cells are all identical (a perfect periodic wire)."""
    r = rng(seed)
    x = r.standard_normal((b, b)) + 1j * r.standard_normal((b, b))
    cell = (x + x.conj().T) / (2.0 * math.sqrt(b))
    cpl = cgauss(r, (b, b), coupling_std)
    H_diag = np.ascontiguousarray(np.broadcast_to(cell, (nb, b, b)))
    H_upper = np.ascontiguousarray(np.broadcast_to(cpl, (nb - 1, b, b)))
    return BTDevice(H_diag, H_upper, name="periodic_wire")


# --------------------------------------------------------------------------
# Nano-ribbon-like slab devices
# --------------------------------------------------------------------------

ORBITALS_PER_ATOM = 10
SLAB_NY = 4
CUTOFF2 = 2  # squared neighbour cutoff on the unit cubic lattice (d <= sqrt(2))


def slab_geometry(b: int):
    """Atom positions (y, z) of one transport cell and the orbital->atom map.

    One atomic layer per cell in the transport direction x, SLAB_NY rows in
    y and nz = ceil(n_atoms / SLAB_NY) columns in z on a unit simple-cubic
    lattice; orbital o belongs to atom o // 10, so the last atom may carry
    fewer than 10 orbitals.  For b = 512 this is the 1 x 4 x 13 slab of 52
    atoms.
    """
    n_atoms = (b + ORBITALS_PER_ATOM - 1) // ORBITALS_PER_ATOM
    nz = (n_atoms + SLAB_NY - 1) // SLAB_NY
    pos = np.array([(a // nz, a % nz) for a in range(n_atoms)], dtype=np.int64)
    atom_of = np.arange(b) // ORBITALS_PER_ATOM
    return pos, atom_of, nz


def _slab_patterns(b: int):
    """Distance matrices (orbital x orbital) within a cell and to the next cell.

    Returns (d_intra, d_inter, d_trans); entries are the interatomic distance
    where the pair is within the cutoff and +inf elsewhere.  ``d_trans``
    couples a cell to its transverse periodic image along z.
    """
    pos, atom_of, nz = slab_geometry(b)
    dy = pos[:, None, 0] - pos[None, :, 0]
    dz = pos[:, None, 1] - pos[None, :, 1]
    r2_intra = dy * dy + dz * dz
    r2_inter = r2_intra + 1                     # neighbouring cell, dx = 1
    dz_img = pos[:, None, 1] - (pos[None, :, 1] + nz)   # transverse image, dz shifted by nz
    r2_trans = dy * dy + dz_img * dz_img

    def to_orb(r2):
        d = np.where(r2 <= CUTOFF2, np.sqrt(r2.astype(np.float64)), np.inf)
        return d[np.ix_(atom_of, atom_of)]

    return to_orb(r2_intra), to_orb(r2_inter), to_orb(r2_trans)


def _draw_cell(r, d_intra, b):
    """One Hermitian on-site block with hoppings std 0.5 e^{-d} and U(-2,2) diagonal."""
    mask = np.isfinite(d_intra)
    amp = np.where(mask, 0.5 * np.exp(-np.where(mask, d_intra, 0.0)), 0.0)
    x = cgauss(r, (b, b), 1.0) * amp
    h = np.triu(x, 1)
    h = h + h.conj().T
    h[np.diag_indices(b)] = r.uniform(-2.0, 2.0, size=b)
    return h


def _draw_coupling(r, d_inter, b):
    mask = np.isfinite(d_inter)
    amp = np.where(mask, 0.5 * np.exp(-np.where(mask, d_inter, 0.0)), 0.0)
    return cgauss(r, (b, b), 1.0) * amp


def _overlap_from_pattern(r, nb, b, mask_d, mask_u, norm):
    """S = I + P, P = norm (K + cI) / (2c), K Hermitian BT on the given pattern.

    c is the largest absolute row sum of K (Gershgorin), so K + cI is PSD and
    ||K + cI||_2 <= 2c, giving 0 <= P and ||P||_2 <= norm.
    """
    Kd = np.empty((nb, b, b), dtype=np.complex128)
    for i in range(nb):
        x = cgauss(r, (b, b), 1.0) * mask_d
        u = np.triu(x, 1)
        Kd[i] = u + u.conj().T + np.diag(r.standard_normal(b)) * np.diag(mask_d)
    Ku = cgauss(r, (nb - 1, b, b), 1.0) * mask_u
    rows = np.abs(Kd).sum(axis=2)
    rows[:-1] += np.abs(Ku).sum(axis=2)
    rows[1:] += np.abs(Ku).sum(axis=1)          # lower blocks are Ku^H: row sums = column sums of Ku
    c = float(rows.max())
    S_diag = np.empty_like(Kd)
    eye = np.eye(b)
    for i in range(nb):
        S_diag[i] = eye + norm * (Kd[i] + c * eye) / (2.0 * c)
    S_upper = norm * Ku / (2.0 * c)
    return np.ascontiguousarray(S_diag), np.ascontiguousarray(S_upper)


def slab_device(nb: int, b: int, seed: int, overlap: float = 0.05) -> BTDevice:
    """Nano-ribbon-like synthetic device (Si ribbon stand-in, Section III).

    b orbitals per cell (10 per atom on a 1 x 4 x nz slab), couplings only
    between atoms within sqrt(2) lattice units, hopping std 0.5 e^{-d},
    on-site energies U(-2, 2), S = I + PSD perturbation of norm ``overlap``
    on the same pattern.  At b = 512 the diagonal blocks are ~14 % dense and
    the coupling blocks ~8.5 %.
    """
    r = rng(seed)
    d_intra, d_inter, _ = _slab_patterns(b)
    H_diag = np.empty((nb, b, b), dtype=np.complex128)
    for i in range(nb):
        H_diag[i] = _draw_cell(r, d_intra, b)
    H_upper = np.empty((nb - 1, b, b), dtype=np.complex128)
    for i in range(nb - 1):
        H_upper[i] = _draw_coupling(r, d_inter, b)
    dev = BTDevice(H_diag, H_upper, name=f"slab{nb}x{b}s{seed}")
    if overlap > 0.0:
        dev.S_diag, dev.S_upper = _overlap_from_pattern(
            r, nb, b, np.isfinite(d_intra), np.isfinite(d_inter), overlap)
    return dev


def slab_lead(b: int, seed: int, overlap: float = 0.05) -> BTDevice:
    """The left lead cell of ``slab_device(2, b, seed)``: a two-block device.

    Returns a 2-block device whose first cell and coupling define a lead
    (cell H_00, S_00; coupling H_01, S_01).
    """
    return slab_device(2, b, seed, overlap)


def scattering_self_energies(dev: BTDevice, seed: int, norm: float = 0.01) -> BTDevice:
    """Attach block-diagonal scattering self-energies to ``dev`` (in place).

    For every block: X = B B^H / ||B B^H||_2 * norm with B complex Gaussian,
    drawn independently for the lesser and the greater component;
    Sigma^< = i X_<, Sigma^> = -i X_>, Sigma^R = (Sigma^> - Sigma^<) / 2.
    Sigma^< and Sigma^> are anti-Hermitian with spectral norm ``norm``, and
    -i Sigma^< and i Sigma^> are positive semi-definite.
    """
    r = rng(seed)
    nb, b = dev.nb, dev.b

    def psd():
        B = cgauss(r, (b, b), 1.0)
        X = B @ B.conj().T
        X = 0.5 * (X + X.conj().T)
        return X * (norm / np.linalg.eigvalsh(X)[-1])

    sl = np.empty((nb, b, b), dtype=np.complex128)
    sg = np.empty((nb, b, b), dtype=np.complex128)
    for i in range(nb):
        sl[i] = 1j * psd()
        sg[i] = -1j * psd()
    dev.sig_l = sl
    dev.sig_g = sg
    dev.sig_r = np.ascontiguousarray(0.5 * (sg - sl))
    return dev


def k_device(dev: BTDevice, seed: int, k: float) -> BTDevice:
    """Transverse-momentum copy of a slab device: H_ii(k) = H_ii + e^{ik} T_i + e^{-ik} T_i^H.

    T_i couples each cell to its transverse periodic image along z (same
    hopping statistics as the slab); it is drawn from ``seed`` and therefore
    identical for every k.  Coupling blocks and S do not depend on k.
    """
    r = rng(seed)
    _, _, d_trans = _slab_patterns(dev.b)
    ph = complex(math.cos(k), math.sin(k))
    H_diag = np.empty_like(dev.H_diag)
    for i in range(dev.nb):
        T = _draw_coupling(r, d_trans, dev.b)
        H_diag[i] = dev.H_diag[i] + ph * T + np.conj(ph) * T.conj().T
    out = dataclasses.replace(dev, H_diag=H_diag, name=f"{dev.name}_k{k:.4f}")
    return out


# Device mix of the batched uneven workload: (b, nb) per device.
DEVICE_MIX = [(128, 20), (256, 40), (384, 60), (512, 80), (640, 20), (768, 40)]


def mixed_devices(seed0: int = 40, scale_nb: float = 1.0, blocks=None):
    """The six devices of the uneven batched workload, seeds seed0..seed0+5."""
    mix = blocks if blocks is not None else DEVICE_MIX
    out = []
    for d, (b, nb) in enumerate(mix):
        nbs = max(2, int(round(nb * scale_nb)))
        out.append(slab_device(nbs, b, seed0 + d))
    return out


def energy_grid(lo: float, hi: float, n: int) -> np.ndarray:
    """Uniform energy grid including both end points."""
    return np.linspace(lo, hi, n, dtype=np.float64)


def boson_bath(nb: int, b: int, n_w: int, k0: int, dE: float, kT: float, strength: float = 0.05,
               width: float = 0.1, decay: float = 2.0):
    """Lesser and greater propagators W^<[k], W^>[k] ([n_w][nb][b][b] complex128) of a bosonic
    bath held in equilibrium at temperature ``kT``, sampled at the frequencies w_k = (k - k0) dE.

    They stand in for the screened interaction (or phonon propagator) of the energy convolution
    of Eq. (3); nothing here is random.  Spatial part, the same in every diagonal block:
    K_oo' = exp(-|o - o'| / decay), real symmetric and positive definite (the exponential
    covariance).  Spectral part: the odd density B(w) = strength (w / width) exp(-w^2 / (2 width^2))
    with the Bose occupation n(w) = 1 / (e^{w / kT} - 1):

        W^<(w) = -i K B(w) n(w),     W^>(w) = -i K B(w) (1 + n(w)),

    both -i K strength kT / width at w = 0 (the limit).  B n >= 0 and B (1 + n) >= 0 for every w,
    W^>(w) = e^{w / kT} W^<(w) (detailed balance) and W^<(w) = W^>(-w).
    """
    if not (kT > 0.0):
        raise ValueError("the bath needs kT > 0")
    o = np.arange(b, dtype=np.float64)
    K = np.exp(-np.abs(o[:, None] - o[None, :]) / decay)
    Wl = np.empty((n_w, nb, b, b), dtype=np.complex128)
    Wg = np.empty((n_w, nb, b, b), dtype=np.complex128)
    for k in range(n_w):
        w = (k - k0) * dE
        if w == 0.0:
            lo = hi = strength * kT / width
        else:
            dens = strength * (w / width) * math.exp(-0.5 * (w / width) ** 2)
            # n and 1 + n = -1 / (e^{-w/kT} - 1), each without cancellation
            lo, hi = dens / math.expm1(w / kT), -dens / math.expm1(-w / kT)
        Wl[k] = (-1j * lo) * K
        Wg[k] = (-1j * hi) * K
    return Wl, Wg
