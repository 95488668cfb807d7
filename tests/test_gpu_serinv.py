"""GPU parity of the partitioned selected inversion (negf_serinv_lesser_greater)
against the oracle at energies where the oracle is stable to the plain bar
(helpers.plain_reference re-checks it), for every partition count the layouts
allow, both complex-product forms, with S != I and scattering self-energies;
and its outputs next to the plain RGF call on the same inputs."""
import numpy as np
import pytest

import workloads as w
from helpers import plain_reference, record
from oracle import rgf as orgf

pytestmark = pytest.mark.gpu

PLAIN_TOL = 1e-10
NAMES = ["GR_diag", "GR_upper", "GR_lower", "GL_diag", "GL_upper", "GG_diag", "GG_upper"]


@pytest.fixture(scope="module")
def nb():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2602_03438_amd import binding
    binding.lib()
    return binding


def _compare(nb, dev, energies, parts, names, greater, cmul, test):
    prob = nb.Problem(nb.DeviceOnGPU(dev), energies, eta=1e-8, mu_l=0.1, mu_r=-0.1, kT=0.025)
    out = nb.serinv_lesser_greater(prob, parts, opts=nb.make_options(cmul=cmul), greater=greater)
    assert np.all(out["info"].cpu().numpy() == 0)
    for k, E in enumerate(energies):
        ref, spread = plain_reference(lambda: orgf.solve_point(dev, E, 1e-8, 0.1, -0.1, 0.025, greater=greater), names)
        for name in names:
            g = out[name][0][k].cpu().numpy()
            r = getattr(ref, name)
            err = float(np.linalg.norm(g - r) / np.linalg.norm(r))
            record(test, E, name, err, PLAIN_TOL, spread[name], None, partitions=parts)
            print(f"  {test} P={parts} E={E:+.3f} {name}: error {err:.3e}", flush=True)
            assert err <= PLAIN_TOL, (parts, E, name, err)
    return out


@pytest.mark.parametrize("cmul", [4, 3])
@pytest.mark.parametrize("parts", [2, 3])
def test_serinv_scattering_slab(nb, parts, cmul):
    dev = w.slab_device(8, 64, 2)
    w.scattering_self_energies(dev, 3)
    _compare(nb, dev, np.array([-0.7, -0.5, 0.5]), parts, NAMES, True, cmul, f"serinv_scattering_cmul{cmul}")


@pytest.mark.parametrize("parts", [2, 3, 4, 5])
def test_serinv_partition_counts(nb, parts):
    """14 blocks: periods 8, 5, 4 and 3 (last partition 6, 4, 2 and 2 interior blocks), on a
    device with scattering self-energies (without broadening inside the device an isolated
    interior at a real energy is nearly singular and the partitioned elimination loses
    accuracy: on this device, ballistic, up to 9e-11 against the plain 1e-10)."""
    dev = w.scattering_self_energies(w.slab_device(14, 32, 5), 6)
    _compare(nb, dev, np.array([-1.4, -0.9, 0.3, 1.3]), parts, NAMES[:5], False, 3, "serinv_partition_counts")


def test_serinv_next_to_rgf(nb):
    """Same inputs through both solvers: every output within the plain bar of the other."""
    dev = w.slab_device(12, 40, 9)
    E = np.array([1.1, -1.4, 0.4, 0.8])
    prob = nb.Problem(nb.DeviceOnGPU(dev), E, eta=1e-8, mu_l=0.1, mu_r=-0.1, kT=0.025)
    a = nb.rgf_lesser_greater([prob], greater=True)
    b = nb.serinv_lesser_greater(prob, 3, greater=True)
    for key in NAMES:
        x, y = a[key][0].cpu().numpy(), b[key][0].cpu().numpy()
        for k in range(E.size):
            assert np.linalg.norm(x[k] - y[k]) <= PLAIN_TOL * np.linalg.norm(x[k]), (key, k)


def test_serinv_rejects_bad_layouts(nb):
    dev = w.slab_device(6, 16, 2)
    prob = nb.Problem(nb.DeviceOnGPU(dev), np.array([0.1]), eta=1e-8)
    with pytest.raises(nb.NegfError):
        nb.serinv_lesser_greater(prob, 1)
    with pytest.raises(nb.NegfError):
        nb.serinv_lesser_greater(prob, 3)      # period 3 leaves the last partition no interior block
