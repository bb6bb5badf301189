"""Writes the stored expected values of the 256 x 256 mixed-tau statistics
workload (tests/test_gpu_config2.py) from the oracle package only:

- config2_theory.json: the linear-response prediction (per-wavevector
  discrete Lyapunov equation of oracle.theory, Sec. II eqs. (11)-(14)
  without the k = 0 restriction) of the site covariance <df_i df_j>, the
  moment covariance in the f-norm at u0 (eq. (23)) and the structure
  factors S_k(rho), S_k(j~_x), S_k(j~_y), R_k (eqs. (24)-(26)) averaged over
  wavevector bands;
- config2_oracle.json: the FP64 oracle's own statistics, 256 x 256, Philox
  seed 2 (independent of the seed-1 GPU runs it is compared with), 2e4
  steps from the equilibrium start, then 1e4 steps sampled every step
  (time blocks of 500).

Workload: rho0 = 1, u0 = (u, 0) for u in {0, 0.1, 0.2}, kT = 1e-4, the six
relaxation times of paper_1204_6734_amd.inputs.mixed_taus(2).

    python tests/golden/make_config2.py [--threads 8] [--skip-oracle]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle import theory as T  # noqa: E402
from paper_1204_6734_amd import inputs as I  # noqa: E402

N = 256
KT = 1e-4
U0 = (0.0, 0.1, 0.2)
SK_KEYS = ("rho", "jx", "jy", "jxjy_re")


def params(ux0, seed, **kw):
    return O.make_params(N, N, rho0=1.0, ux0=ux0, kT=KT, tau=I.mixed_taus(2), seed=seed, **kw)


def theory(ux0):
    p = params(ux0, 1)
    ck = T.k_covariances(p)
    C = T.site_covariance(p, ck)
    Cm = T.moment_covariance(p, C)
    sk = T.structure_factors(p, ck)
    plane = T.band_masks(N, N)
    axis = T.band_masks(N, N, T.AXIS_EDGES, axis=True)
    return {"cov_f": C.ravel().tolist(), "cov_m": Cm.ravel().tolist(),
            "sk_plane": {k: T.band_means(sk[k], plane).tolist() for k in SK_KEYS},
            "sk_axis": {k: T.band_means(sk[k], axis).tolist() for k in SK_KEYS}}


def oracle_stats(ux0):
    L = O.Lattice(params(ux0, 2, sample_every=1, block_steps=500))
    L.step(20000)
    L.reset_stats()
    L.step(10000)
    c = L.covariance()
    out = {k: np.asarray(c[k]).ravel().tolist()
           for k in ("mean_df", "cov_f", "se_cov_f", "cov_m_fnorm_u0", "se_cov_m")}
    out["nsamples"] = c["nsamples"]
    out["nblocks"] = c["nblocks"]
    L.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--skip-oracle", action="store_true")
    a = ap.parse_args()
    O.set_threads(a.threads)
    meta = {"nx": N, "ny": N, "kT": KT, "tau": list(I.mixed_taus(2)), "u0": list(U0)}
    th = {"meta": dict(meta, plane_edges=list(T.PLANE_EDGES), axis_edges=list(T.AXIS_EDGES))}
    for u in U0:
        t0 = time.time()
        th[f"{u:g}"] = theory(u)
        print(f"theory u0={u}: {time.time() - t0:.1f} s", flush=True)
    with open(os.path.join(HERE, "config2_theory.json"), "w") as fh:
        json.dump(th, fh, indent=0)
    if a.skip_oracle:
        return
    orc = {"meta": dict(meta, seed=2, therm_steps=20000, sampled_steps=10000,
                        block_steps=500)}
    for u in U0:
        t0 = time.time()
        orc[f"{u:g}"] = oracle_stats(u)
        print(f"oracle u0={u}: {time.time() - t0:.1f} s", flush=True)
        with open(os.path.join(HERE, "config2_oracle.json"), "w") as fh:
            json.dump(orc, fh, indent=0)


if __name__ == "__main__":
    main()
