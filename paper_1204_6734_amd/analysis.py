"""Host-side analysis of GPU runs (after the hot path, on its FP64 readouts).

- ``velocity_sweep``: one ensemble of identical lattices that differ only in
  the background velocity u_x0, advanced in one batched launch per step;
  returns the moment covariances <dM^a dM^b> / (mu rho0) - delta^{ab} per
  velocity, measured in the basis the paper uses for that scheme (the
  Hermite moments for the Hermite norm, the f-norm moments at (rho0, u0)
  otherwise), with time-block standard errors.
- ``lq_maps``: the linear and quadratic coefficients l, q of those
  deviations as functions of u_x0 (the maps of Figs. 7 and 18; a fit of
  l u + q u^2, no constant term, as in the captions of those figures).
- ``structure_factor_maps``: S_k of rho, j~_x, j~_y and the cross
  correlator R_k of eqs. (24)-(26), normalised by mu rho0 so that the ideal
  gas gives S = 1, R = 0 (Figs. 10 and 19-21).

Nothing here computes the method itself: the lattices run through libflb.
"""
from __future__ import annotations

import numpy as np


def noise_strength(kT: float) -> float:
    """mu = kT / theta with theta = 1/3 on D2Q9 (the noise scale of the
    covariance of eq. (16) at temperature kT)."""
    return 3.0 * kT


def velocity_sweep(F, basis: int, us, nx: int = 21, ny: int = 21, kT: float = 1e-5,
                   tau=(1.0,) * 6, therm: int = 3000, steps: int = 60000,
                   block_steps: int = 1000, seed: int = 11, precision=None,
                   graph_chunk: int = 100, rho0: float = 1.0) -> dict:
    """Run every u_x0 in ``us`` as one replica of an ensemble (own seed
    seed + index), thermalise ``therm`` steps from equilibrium, sample every
    step for ``steps`` steps and return {"us", "dev", "se", "nsamples"} with
    dev[n] = <dM dM>(us[n]) / (mu rho0) - I and its standard errors."""
    us = np.asarray(us, dtype=float)
    prec = F.FP64 if precision is None else precision
    ps = [F.make_params(nx, ny, rho0=rho0, ux0=float(u), kT=kT, tau=tau, seed=seed + k,
                        basis=basis, precision=prec, sample_every=1, block_steps=block_steps)
          for k, u in enumerate(us)]
    E = F.Ensemble(ps, graph_chunk=graph_chunk)
    E.step(therm)
    E.reset_stats()
    E.step(steps)
    mu_rho = noise_strength(kT) * rho0
    key, sekey = (("cov_m_hermite", "se_cov_m_hermite") if basis == F.BASIS_HERMITE
                  else ("cov_m_fnorm_u0", "se_cov_m"))
    dev, se = [], []
    nsamples = 0
    for k in range(len(us)):
        c = E.covariance(k)
        dev.append(c[key] / mu_rho - np.eye(9))
        se.append(c[sekey] / mu_rho)
        nsamples = c["nsamples"]
    E.close()
    return {"us": us, "dev": np.array(dev), "se": np.array(se), "nsamples": nsamples}


def lq_maps(us, dev, se=None):
    """Fit dev_ab(u) = l_ab u + q_ab u^2 for every (a, b) (weighted by 1/se^2
    when standard errors are given).  Returns l, q (9 x 9) and, with se, their
    standard errors sl, sq."""
    us = np.asarray(us, dtype=float)
    dev = np.asarray(dev, dtype=float)
    X = np.stack([us, us ** 2], axis=1)
    l = np.zeros((9, 9))
    q = np.zeros((9, 9))
    sl = np.full((9, 9), np.nan)
    sq = np.full((9, 9), np.nan)
    for a in range(9):
        for b in range(9):
            y = dev[:, a, b]
            if se is None:
                coef, *_ = np.linalg.lstsq(X, y, rcond=None)
                l[a, b], q[a, b] = coef
                continue
            w = 1.0 / np.maximum(np.asarray(se)[:, a, b], 1e-300)
            Xw = X * w[:, None]
            coef, *_ = np.linalg.lstsq(Xw, y * w, rcond=None)
            l[a, b], q[a, b] = coef
            cov = np.linalg.inv(Xw.T @ Xw)
            sl[a, b], sq[a, b] = np.sqrt(np.diag(cov))
    if se is None:
        return l, q
    return l, q, sl, sq


def structure_factor_maps(L, kT: float, rho0: float = 1.0) -> dict:
    """S_k(rho~), S_k(j~_x), S_k(j~_y) and R_k (complex) of a lattice that
    sampled structure factors, divided by mu rho0; arrays are [ky][kx]."""
    mu_rho = noise_strength(kT) * rho0
    out = {name: L.structure_factor(w) / mu_rho
           for name, w in (("rho", 0), ("jx", 1), ("jy", 2))}
    out["R"] = (L.structure_factor(3) + 1j * L.structure_factor(4)) / mu_rho
    return out
