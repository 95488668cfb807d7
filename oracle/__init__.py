"""CPU oracle for the NEGF hot path -- TEST INFRASTRUCTURE ONLY.

This package is the slow, obviously-correct reference that the GPU library is
checked against.  Only the test suite, the smoke check of the entry module
and the CPU-baseline leg of the benchmark may import it.  The product path
never calls it and shares no code with it; the two meet only in the seeded
input generators of ``workloads``.

Everything here is plain NumPy in complex128 / float64 with LAPACK through
``numpy.linalg``.  Each function states the passage of the paper (Eq. (1),
Eq. (2), Section II) or the textbook method it follows.

Modules
  leads       -- open-boundary self-energies (Sancho-Rubio decimation)
  dense       -- brute-force dense inversion: the definition of Eq. (1)/(2)
  rgf         -- recursive Green's function selected inversion (Section II)
  observables -- current, density of states
  emulate     -- the FP32-product / FP64-refinement variant, emulated with
                 complex64 NumPy products (diagnostic only)
  mlp         -- float64 reference of the small MLP used to seed the lead
                 iteration, with a hand-written backward pass and Adam
  econv       -- the energy convolution of Eq. (3) on a uniform grid (the
                 plain sum), and the (E; i,j) -> (i,j; E) layout change
  scba        -- the self-consistent loop of Fig. 1 around Eq. (1)-(3) with a
                 fixed boson bath (solve, convolve, mix, repeat)

Parity status: every function is pinned by the CPU tests against closed
forms, brute force or physical invariants, except the absolute throughput,
for which the paper prints no number (parity unpinned).
"""
from . import leads, dense, rgf, observables, emulate, mlp, econv, scba  # noqa: F401
