"""Pins of the energy-convolution oracle (oracle/econv.py) against what the
mathematics fixes: the identity kernel, shifts, a library routine for the
full linear convolution, a closed form for geometric sequences, linearity and
the layout change being a pure relabelling; plus planted mistakes."""
import os
import types

import numpy as np
import pytest

from oracle import econv

ORACLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "econv.py")


def _rand(r, shape):
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def _pins(mod):
    r = np.random.Generator(np.random.PCG64(5))
    ok = {}
    G = _rand(r, (37, 5))
    # identity kernel: W = delta at k0 -> B = scale G
    for k0 in (0, 3, 6):
        W = np.zeros((7, 5), complex)
        W[k0] = 1.0
        ok[f"delta{k0}"] = np.allclose(mod.energy_convolution(G, W, k0, 2.5 - 1j), (2.5 - 1j) * G, atol=1e-14)
    # a delta away from k0 shifts the series by (k - k0), with zeros entering at the edge
    W = np.zeros((7, 5), complex)
    W[5] = 1.0
    B = mod.energy_convolution(G, W, 2)
    ok["shift"] = np.allclose(B[3:], G[:-3], atol=1e-14) and np.allclose(B[:3], 0)
    # library routine: the slice [k0, k0 + n_e) of numpy's full linear convolution
    W = _rand(r, (11, 5))
    B = mod.energy_convolution(G, W, 4)
    ref = np.stack([np.convolve(G[:, x], W[:, x])[4:4 + 37] for x in range(5)], axis=1)
    ok["convolve"] = np.allclose(B, ref, atol=1e-12)
    # closed form: G[e] = a^e, W[k] = c^k (one element); for 0 <= e + k0 - k < n_e the sum is geometric
    a, c, n_e, n_w, k0 = 0.9 + 0.1j, 0.7 - 0.2j, 20, 9, 4
    Ge = (a ** np.arange(n_e))[:, None]
    Wk = (c ** np.arange(n_w))[:, None]
    B = mod.energy_convolution(Ge, Wk, k0)[:, 0]
    ref = np.zeros(n_e, complex)
    for e in range(n_e):
        klo, khi = max(0, e + k0 - n_e + 1), min(n_w - 1, e + k0)
        q = c / a
        ref[e] = a ** (e + k0) * (q ** klo - q ** (khi + 1)) / (1 - q)
    ok["geometric"] = np.allclose(B, ref, rtol=1e-12, atol=1e-14)
    # linear in each argument
    G2 = _rand(r, (37, 5))
    ok["linear"] = np.allclose(mod.energy_convolution(G + 2 * G2, W, 4),
                               mod.energy_convolution(G, W, 4) + 2 * mod.energy_convolution(G2, W, 4), atol=1e-12)
    X = _rand(r, (6, 4))
    T = mod.to_element_major(X)
    ok["transpose"] = T.shape == (4, 6) and all(T[j, i] == X[i, j] for i in range(6) for j in range(4))
    return ok


def test_oracle_pins():
    ok = _pins(econv)
    assert all(ok.values()), ok


MUTATIONS = [
    ("shift = k0 - k", "shift = k - k0"),
    ("hi = min(n_e, n_e - shift)", "hi = min(n_e, n_e - shift) - 1"),
    ("B[lo:hi] += G[lo + shift:hi + shift] * W[k]", "B[lo:hi] += G[lo + shift:hi + shift] * W[k].conj()"),
    ("return scale * B", "return B"),
    ("return np.ascontiguousarray(np.swapaxes(X, 0, 1))", "return np.ascontiguousarray(X.reshape(X.shape[1], -1))"),
]


@pytest.mark.parametrize("k", range(len(MUTATIONS)))
def test_planted_mistake_is_caught(k):
    old, new = MUTATIONS[k]
    src = open(ORACLE).read()
    assert old in src
    mod = types.ModuleType("econv_variant")
    exec(compile(src.replace(old, new, 1), "<econv variant>", "exec"), mod.__dict__)
    with np.errstate(all="ignore"):
        try:
            ok = _pins(mod)
        except (ValueError, IndexError):
            return
    assert not all(ok.values()), (new, ok)
