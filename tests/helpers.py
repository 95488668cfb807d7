"""Shared helpers of the test suite."""
import numpy as np

from oracle import leads


def well_posed(dev, energies, eta=1e-8, min_ratio=1e-2):
    """Energies at which both leads carry propagating modes.

    Where ||Gamma|| << ||Sigma^R|| (an energy in or at the edge of a lead gap)
    Gamma = i (Sigma - Sigma^H) is a cancellation of nearly equal numbers, G^<
    is O(eta) and its relative error is set by that cancellation, not by the
    solver: such points are ill-posed for a relative comparison of G^<.
    """
    keep = []
    for E in energies:
        ok = True
        for side in (0, 1):
            r = leads.lead_self_energy(dev, side, E, eta)
            ok &= np.linalg.norm(r.gamma) > min_ratio * np.linalg.norm(r.sigma_r)
        if ok:
            keep.append(E)
    return np.array(keep)


class refined_inversions:
    """Context in which every numpy.linalg.inv (used by the oracle) is followed
    by Newton refinement steps X <- X + X (I - M X).  The change this makes to
    an oracle result measures the result's sensitivity to rounding in the
    inversions; at energies where the decimation at small eta is
    ill-conditioned that sensitivity exceeds 1e-10 for any double-precision
    method."""

    def __init__(self, steps=2):
        self.steps = steps

    def __enter__(self):
        import numpy.linalg as la
        self._orig = la.inv
        orig = self._orig
        steps = self.steps

        def inv(m):
            x = orig(m)
            eye = np.eye(m.shape[-1])
            for _ in range(steps):
                x = x + x @ (eye - m @ x)
            return x

        la.inv = inv
        import oracle.rgf as orgf_mod
        self._orig_rgf = orgf_mod.inv
        orgf_mod.inv = inv
        return self

    def __exit__(self, *exc):
        import numpy.linalg as la
        import oracle.rgf as orgf_mod
        la.inv = self._orig
        orgf_mod.inv = self._orig_rgf
        return False


def point_tolerance(compute, names, base=1e-10, factor=4.0):
    """(reference, {name: tolerance}) for one oracle evaluation ``compute()``:
    tolerance = max(base, factor * change of the result under refined inversions)."""
    ref = compute()
    with refined_inversions():
        ref2 = compute()
    tol = {}
    for n in names:
        a, b = getattr(ref, n), getattr(ref2, n)
        spread = float(np.linalg.norm(a - b) / np.linalg.norm(a))
        tol[n] = max(base, factor * spread)
    return ref, tol
