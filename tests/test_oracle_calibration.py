"""Calibration of the oracle's error bars and of its thermal start (CPU).

Every statistical comparison in the test suite ("within N standard errors")
divides by the time-block standard error the oracle (and the library, which
computes the same estimator) reports.  These tests pin that error bar to
something other than its own formula: the spread of the same estimate over
independent noise realisations.  Sec. III's run protocol (thermalise, then
average over time) is what the blocking estimator summarises; with blocks
much longer than the correlation time of the slowest mode, the variance of
a run's covariance estimate across seeds equals the mean squared standard
error the runs report.

Pinned here:
- D2Q9, 16 x 16, u0 = 0 and (0.15, 0), tau = 1: 32 seeds, 10^4 sampled steps
  in 20 blocks of 500 each; per correlator the ratio of the across-seed
  variance to the mean reported SE^2, averaged over the 45 unique entries,
  lies in [0.7, 1.4] (a standard error twice too large gives 0.25, one too
  small by sqrt 2 gives 2);
- D3Q19, 4^3, u0 = 0: the same with 32 seeds of 1000 steps in 20 blocks;
- the thermal start (the ideal-gas state of eq. (16) with mu = 3 kT): over
  a 256 x 256 lattice, per-site deviations from f^0(rho0, u0) have mean 0
  and covariance mu f^0_i delta_ij within the sampling error of 65536 sites
  (a wrong amplitude, e.g. kT instead of 3 kT, misses by ~100 standard
  errors).
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
from oracle import d3q19 as D

# the oracle's C calls release the GIL, so threads run the seeds in parallel
WORKERS = 8


def _ratio(covs, ses, n):
    """Per unique entry: across-seed variance of the estimate over the mean
    squared reported standard error."""
    C = np.array(covs)
    S = np.array(ses)
    iu = np.triu_indices(n)
    var = C.var(axis=0, ddof=1)[iu]
    se2 = (S ** 2).mean(axis=0)[iu]
    return var / se2


@pytest.mark.parametrize("ux0", [0.0, 0.15])
def test_d2q9_blocking_standard_error_matches_seed_spread(ux0):
    def run(seed):
        L = O.Lattice(O.make_params(16, 16, ux0=ux0, kT=1e-4, seed=seed, sample_every=1,
                                    block_steps=500))
        L.step(10000)
        c = L.covariance()
        L.close()
        return c

    with ThreadPoolExecutor(WORKERS) as ex:
        cs = list(ex.map(run, range(100, 132)))
    assert all(c["nblocks"] == 20 for c in cs)
    r = _ratio([c["cov_f"] for c in cs], [c["se_cov_f"] for c in cs], 9)
    rm = _ratio([c["cov_m_fnorm_u0"] for c in cs], [c["se_cov_m"] for c in cs], 9)
    # the moment covariances whose true variance vanishes (the conserved
    # rho, j rows: mass and momentum are exactly constant) are left out
    keep = np.triu_indices(9)
    live = [(a >= 3 and b >= 3) for a, b in zip(*keep)]
    rm = rm[np.array(live)]
    print(f"u0 {ux0}: var/SE^2 cov_f mean {r.mean():.3f} median {np.median(r):.3f}; "
          f"cov_m mean {rm.mean():.3f} median {np.median(rm):.3f}")
    for x in (r, rm):
        assert 0.7 <= x.mean() <= 1.4, x.mean()
        assert 0.6 <= np.median(x) <= 1.5, np.median(x)


def test_d3q19_blocking_standard_error_matches_seed_spread():
    def run(seed):
        L = D.Lattice(D.make_params(4, 4, 4, kT=1e-4, seed=seed, sample_every=1,
                                    block_steps=50))
        L.step(1000)
        c = L.covariance()
        return c

    with ThreadPoolExecutor(WORKERS) as ex:
        cs = list(ex.map(run, range(200, 232)))
    assert all(c["nblocks"] == 20 for c in cs)
    r = _ratio([c["cov_f"] for c in cs], [c["se_cov_f"] for c in cs], 19)
    print(f"D3Q19: var/SE^2 mean {r.mean():.3f} median {np.median(r):.3f}")
    assert 0.7 <= r.mean() <= 1.4, r.mean()
    assert 0.6 <= np.median(r) <= 1.5, np.median(r)


@pytest.mark.parametrize("ux0,uy0", [(0.0, 0.0), (0.1, 0.05)])
def test_thermal_start_has_ideal_gas_covariance(ux0, uy0):
    n, kT = 256, 1e-3
    mu = 3 * kT
    L = O.Lattice(O.make_params(n, n, ux0=ux0, uy0=uy0, kT=kT, seed=5, init=O.INIT_THERMAL))
    f0 = O.equilibrium(1.0, ux0, uy0)
    df = (L.populations() - f0[:, None, None]).reshape(9, -1)
    N = df.shape[1]
    want = mu * np.diag(f0)
    sig = np.sqrt(mu * f0)
    # sampling errors of the mean, the variances and the cross products of
    # independent Gaussians
    z_mean = df.mean(axis=1) / (sig / np.sqrt(N))
    C = df @ df.T / N
    se = np.outer(sig, sig) / np.sqrt(N)
    se[np.diag_indices(9)] *= np.sqrt(2.0)
    z = (C - want) / se
    print(f"thermal start u0=({ux0},{uy0}): max|z| cov {np.abs(z).max():.2f}, "
          f"mean {np.abs(z_mean).max():.2f}")
    assert np.abs(z_mean).max() < 4.5
    assert np.abs(z).max() < 4.5
    assert 0.5 < np.sqrt((z ** 2).mean()) < 1.6
