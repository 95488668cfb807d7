"""Host-side preprocessing of the learned lead initialiser (no GPU)."""
import numpy as np

import workloads as w
from oracle import leads


def test_lead_basis_is_s_orthonormal_and_features_shape():
    from paper_2602_03438_amd import learned
    dev = w.slab_device(2, 40, 3)
    bs = learned.lead_basis(dev, 0)
    U, S0 = bs.U, bs.S0
    assert np.allclose(U.conj().T @ S0 @ U, np.eye(40), atol=1e-12)
    assert np.allclose(dev.H_diag[0] @ U, S0 @ U @ np.diag(bs.lam), atol=1e-10)
    X = learned.features(bs, np.array([0.1, -0.4]))
    assert X.shape == (80, learned.N_FEAT) and X.dtype == np.float32
    assert np.allclose(X[:40, 0], 0.1) and np.allclose(X[40:, 1], -0.4 - bs.lam, atol=1e-6)


def test_eigenbasis_representation_exact_without_coupling():
    """With no inter-cell coupling g_s = (z S0 - H0)^{-1} is diagonal in the eigenbasis,
    so the per-mode target/seed transform reproduces it exactly."""
    from paper_2602_03438_amd import learned
    dev = w.slab_device(2, 24, 5)
    dev.H_upper[:] = 0.0
    dev.S_upper[:] = 0.0
    bs = learned.lead_basis(dev, 0)
    z = complex(0.3, 1e-3)
    g = np.linalg.inv(z * bs.S0 - dev.H_diag[0])
    x = np.diag(bs.U.conj().T @ bs.S0 @ g @ bs.S0 @ bs.U)
    g_seed = bs.U @ np.diag(x) @ bs.U.conj().T
    assert np.allclose(g_seed, g, atol=1e-10)
    assert np.allclose(x, 1.0 / (z - bs.lam), atol=1e-10)
    # and the decimation oracle agrees that such a lead has g_s = (z S0 - H0)^{-1}
    r = leads.lead_self_energy(dev, 0, 0.3, 1e-3)
    assert np.allclose(r.g_surf, g, atol=1e-10)
