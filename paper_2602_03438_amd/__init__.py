"""MI355X-native hot path of atomistic NEGF: RGF selected inversion of the
block-tridiagonal system E S - H - Sigma (Eq. (1) and Eq. (2) of the paper)
with Sancho-Rubio lead self-energies, as hand-written HIP kernels for gfx950
behind a C ABI (include/negf.h, libnegf.so).

``paper_2602_03438_amd.binding`` is the ctypes layer; importing this package
does not load the library or torch.
"""
__all__ = ["binding", "build"]
