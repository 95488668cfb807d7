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
