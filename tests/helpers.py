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


def oracle_spread(compute, names):
    """(reference, {name: spread}) for one oracle evaluation ``compute()``: the
    spread of an output is its relative change when every inversion of the
    oracle is followed by Newton refinement, i.e. how far rounding in the
    inversions alone moves the oracle's own answer at this point."""
    ref = compute()
    with refined_inversions():
        ref2 = compute()
    spread = {}
    for n in names:
        a, b = getattr(ref, n), getattr(ref2, n)
        spread[n] = float(np.linalg.norm(a - b) / np.linalg.norm(a))
    return ref, spread


# Where factor * spread <= the plain bar, the oracle is stable enough to referee
# the plain double-precision bar itself.
SPREAD_FACTOR = 4.0


def point_tolerance(compute, names, base=1e-10, factor=SPREAD_FACTOR):
    """(reference, {name: tolerance}) for one oracle evaluation ``compute()``:
    tolerance = max(base, factor * spread) (see oracle_spread).  Used by the
    tests named ``..._conditioned``, at points where the oracle itself is not
    stable to the plain bar."""
    ref, spread = oracle_spread(compute, names)
    return ref, {n: max(base, factor * spread[n]) for n in names}


def plain_reference(compute, names, bar=1e-10, factor=SPREAD_FACTOR):
    """(reference, spreads) at a point where the plain bar applies unchanged:
    asserts that the oracle is stable there (factor * spread <= bar for every
    output), so that the bar measures the GPU path and not the conditioning."""
    ref, spread = oracle_spread(compute, names)
    bad = {n: s for n, s in spread.items() if factor * s > bar}
    assert not bad, f"oracle not stable to the plain bar at this point: spreads {bad}"
    return ref, spread


def kappa_proxy(dev, ref):
    """Conditioning proxy of one point: max over block rows of the summed
    Frobenius norms of the A blocks in the row, times max_i ||G_ii||_F."""
    from oracle import rgf as orgf
    Ad, Au, _ = orgf.assemble_blocks(dev, ref.E, ref.lead_l.sigma_r, ref.lead_r.sigma_r)
    nb = len(Ad)
    rows = []
    for i in range(nb):
        r = np.linalg.norm(Ad[i])
        if i < nb - 1:
            r += np.linalg.norm(Au[i])
        if i > 0:
            r += np.linalg.norm(Au[i - 1])
        rows.append(r)
    return float(max(rows) * max(np.linalg.norm(g) for g in ref.GR_diag))


# ---- per-point parity records -------------------------------------------------
# Every GPU parity comparison appends (test, point, output kind, error, bar,
# oracle spread, conditioning proxy); at its end the session writes them to
# parity/records.jsonl under the results folder (conftest.py) so that a run
# states which bar each point was held to.
RECORDS = []


def record(test, E, name, err, bar, spread=None, kappa=None, **extra):
    RECORDS.append(dict(test=test, E=float(E), name=name, err=float(err), bar=float(bar),
                        spread=None if spread is None else float(spread),
                        kappa=None if kappa is None else float(kappa), **extra))
