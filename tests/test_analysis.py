"""Host-side analysis helpers (no GPU): the l/q fits recover known
polynomials and the normalising equilibrium is eq. (A1)."""
import numpy as np

import oracle as O
from paper_1204_6734_amd import analysis as A

US = np.round(np.arange(-0.25, 0.2501, 0.05), 10)


def test_lq_maps_recover_known_coefficients():
    rng = np.random.default_rng(1)
    l0 = rng.normal(size=(9, 9))
    q0 = rng.normal(size=(9, 9))
    dev = np.array([l0 * u + q0 * u * u for u in US])
    l, q = A.lq_maps(US, dev)
    assert np.abs(l - l0).max() < 1e-12 and np.abs(q - q0).max() < 1e-12
    se = np.full_like(dev, 1e-3)
    l2, q2, sl, sq = A.lq_maps(US, dev, se)
    assert np.abs(l2 - l0).max() < 1e-12 and np.abs(q2 - q0).max() < 1e-12
    # standard errors of a weighted straight fit: (X^T W X)^-1 on the diagonal
    X = np.stack([US, US ** 2], axis=1) / 1e-3
    cov = np.linalg.inv(X.T @ X)
    assert abs(sl[0, 0] - np.sqrt(cov[0, 0])) < 1e-12 and abs(sq[4, 4] - np.sqrt(cov[1, 1])) < 1e-12


def test_equilibrium_is_eq_A1():
    for rho, ux, uy in [(1.0, 0.0, 0.0), (1.3, 0.1, -0.2), (0.7, 0.25, 0.05)]:
        assert np.abs(A.equilibrium(rho, ux, uy) - O.equilibrium(rho, ux, uy)).max() < 1e-15


def test_noise_strength():
    assert abs(A.noise_strength(1e-4) - 3e-4) < 1e-18
