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
- ``mixed_tau_statistics``: one long run of a lattice with the statistics
  of Sec. IV switched on (moment covariances every step, structure factors
  every few steps), with the structure factors kept per time segment so
  that their standard errors can be formed by blocking.

Nothing here computes the method itself: the lattices run through libflb.
"""
from __future__ import annotations

import time

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
    dev, se, cov_f, se_f = [], [], [], []
    nsamples = 0
    for k in range(len(us)):
        c = E.covariance(k)
        dev.append(c[key] / mu_rho - np.eye(9))
        se.append(c[sekey] / mu_rho)
        cov_f.append(c["cov_f"] / noise_strength(kT))
        se_f.append(c["se_cov_f"] / noise_strength(kT))
        nsamples = c["nsamples"]
    E.close()
    return {"us": us, "dev": np.array(dev), "se": np.array(se), "cov_f": np.array(cov_f),
            "se_f": np.array(se_f), "nsamples": nsamples}


def equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    """f_i^0(rho, u) of eq. (A1) on the D2Q9 set (for normalising results)."""
    vx = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], float)
    vy = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], float)
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    cu = vx * ux + vy * uy
    return w * rho * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * (ux * ux + uy * uy))


def paper_experiments(F, kT: float = 1e-6 / 3, therm: int = 100_000, steps: int = 1_000_000,
                      sk_steps: int = 200_000, sk_every: int = 10) -> dict:
    """The paper's 21 x 21 experiments on the GPU (Secs. III and IV): the
    noise strength of its rho0 = 1e6 (mu / rho0 = 1e-6), u_x0 = -0.25 ... 0.25,
    equilibration then sampling every step, for the Hermite norm, the local
    f-norm and the table f-norm.  Returns per scheme the variances of the
    populations against f_i^0 (Figs. 2-4, 12-15), the moment variances (Figs.
    6, 16, 17), the l/q maps and the printed q / l summary (Figs. 7, 18), and
    S_k / R_k deviations at u_x0 = 0, 0.1, 0.2 (Figs. 8-10, 19-21)."""
    us = np.round(np.arange(-0.25, 0.2501, 0.05), 10)
    out = {"kT": kT, "mu_over_rho0": noise_strength(kT), "us": us.tolist(), "steps": steps,
           "therm": therm}
    schemes = (("hermite", F.BASIS_HERMITE), ("fnorm_local", F.BASIS_FNORM_LOCAL),
               ("fnorm_lut", F.BASIS_FNORM_LUT))
    import sys
    for name, basis in schemes:
        print(f"paper experiments: {name} sweep", file=sys.stderr, flush=True)
        r = velocity_sweep(F, basis, us, kT=kT, therm=therm, steps=steps, block_steps=10_000)
        l, q, sl, sq = lq_maps(us, r["dev"], r["se"])
        f0 = np.array([equilibrium(1.0, u, 0.0) for u in us])
        var_f = np.array([np.diag(c) for c in r["cov_f"]])
        res = {
            # <df_i^2> / (mu f_i^0(u0)) - 1 per velocity and direction
            "var_f_over_f0_minus_1": (var_f / f0 - 1).tolist(),
            "var_m_minus_1": [np.diag(d).tolist() for d in r["dev"]],
            "q_diag": np.diag(q).tolist(), "q_diag_se": np.diag(sq).tolist(),
            "l_max_abs": float(np.abs(l).max()),
            "q": {"rho": q[0, 0], "Pi_xx-yy": q[3, 3], "j_y": q[2, 2]},
            "nsamples": int(r["nsamples"]),
        }
        sk = {}
        for u in (0.0, 0.1, 0.2):
            p = F.make_params(21, 21, ux0=u, kT=kT, basis=basis, seed=99, sk_every=sk_every)
            L = F.Lattice(p)
            L.step(therm)
            L.reset_stats()
            L.step(sk_steps)
            m = structure_factor_maps(L, kT)
            mask = np.ones((21, 21), bool)
            mask[0, 0] = False
            sk[f"{u:g}"] = {
                "S_rho_max_dev_kx_axis": float(np.abs(m["rho"][0, 1:] - 1).max()),
                "S_jx_max_dev_kx_axis": float(np.abs(m["jx"][0, 1:] - 1).max()),
                "S_rho_mean_dev": float(np.abs(m["rho"][mask] - 1).mean()),
                "S_jx_mean_dev": float(np.abs(m["jx"][mask] - 1).mean()),
                "R_max_abs": float(np.abs(m["R"][mask]).max()),
            }
            L.close()
        res["structure_factors"] = sk
        out[name] = res
    return out


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


def mixed_tau_statistics(F, precision: int, ux0: float, nx: int = 256, ny: int = 256,
                         kT: float = 1e-4, tau=None, seed: int = 1, therm: int = 20_000,
                         steps: int = 100_000, sk_every: int = 10, segments: int = 20,
                         block_steps: int = 5_000, basis: int = 0) -> dict:
    """A periodic nx x ny lattice at rest density 1 in background flow
    (u_x0, 0): ``therm`` steps from equilibrium, then ``steps`` steps sampling
    the correlators every step (time blocks of ``block_steps``) and the
    structure factors every ``sk_every`` steps.  Returns the library's
    covariance readout ("cov") and the structure factors of each of
    ``segments`` equal time segments ("sk_segments", shape (segments, 5, ny,
    nx): rho, j~_x, j~_y, Re and Im of the cross term, each <|dA(k)|^2> /
    (nx ny)), plus the wall time of the sampled steps."""
    return mixed_tau_statistics_many(F, precision, (ux0,), nx, ny, kT, tau, seed, therm, steps,
                                     sk_every, segments, block_steps, basis)[0]


def mixed_tau_statistics_many(F, precision: int, ux0s, nx: int = 256, ny: int = 256,
                              kT: float = 1e-4, tau=None, seed: int = 1, therm: int = 20_000,
                              steps: int = 100_000, sk_every: int = 10, segments: int = 20,
                              block_steps: int = 5_000, basis: int = 0) -> list:
    """`mixed_tau_statistics` for several background flows at once: one
    lattice per u_x0, each on its own stream, stepped side by side.  A small
    lattice is one wavefront per SIMD, so its step is held by latency;
    lattices on separate streams overlap on the device, and each replays
    captured graphs of whole multiples of ``sk_every`` steps (the sampled
    and structure-factor steps inside them), so the host keeps up.  Every
    lattice computes exactly what it computes alone; "seconds" is the wall
    time of the sampled steps of all of them together."""
    if tau is None:
        from . import inputs
        tau = inputs.mixed_taus(2)
    if therm % sk_every or steps % (segments * sk_every):
        raise ValueError("therm and steps / segments must be multiples of sk_every")
    chunk = 2 * sk_every * max(1, 50 // sk_every)  # even, a multiple of sk_every
    lats = []
    for u in ux0s:
        p = F.make_params(nx, ny, precision=precision, basis=basis, rho0=1.0, ux0=float(u), kT=kT,
                          tau=tau, seed=seed, sample_every=1, block_steps=block_steps,
                          sk_every=sk_every)
        L = F.Lattice(p)
        L.set_graph_chunk(chunk)
        lats.append(L)
    for L in lats:
        L.step(therm)
    for L in lats:
        L.reset_stats()
    seg = steps // segments
    per = seg // sk_every  # structure-factor samples per segment
    sums_prev = [np.zeros((5, ny, nx)) for _ in lats]
    out = [np.empty((segments, 5, ny, nx)) for _ in lats]
    t0 = time.perf_counter()
    for s in range(segments):
        for L in lats:
            L.step(seg)
        for i, L in enumerate(lats):
            sums = np.stack([L.structure_factor(w) for w in range(5)]) * ((s + 1) * per)
            out[i][s] = (sums - sums_prev[i]) / per
            sums_prev[i] = sums
    for L in lats:
        L.sync()
    dt = time.perf_counter() - t0
    res = []
    for i, (L, u) in enumerate(zip(lats, ux0s)):
        res.append({"cov": L.covariance(), "sk_segments": out[i], "seconds": dt, "nx": nx,
                    "ny": ny, "steps": steps, "therm": therm, "ux0": float(u), "kT": kT,
                    "tau": list(tau), "seed": seed, "lattices_together": len(lats)})
        L.close()
    return res
