"""Seeded synthetic workloads (no method arithmetic here).

Every input the tests and the benchmark feed to both the GPU library and the
CPU oracle comes from these generators: parameter draws, initial fields and
request streams.  The paper's own runs are synthetic too (periodic lattices
at rest or in uniform flow, Sec. III); the recipes below follow the
workloads the library is measured on.
"""
from __future__ import annotations

import math

import numpy as np

TAU_ONE = (1.0,) * 6


def mixed_taus(seed: int = 2, low: float = 0.6, high: float = 1.5) -> tuple:
    """Six relaxation times (modes 3..8), one uniform draw each."""
    return tuple(float(x) for x in np.random.default_rng(seed).uniform(low, high, 6))


def shear_wave_fields(nx: int, ny: int, rho0: float = 1.0, ux0: float = 0.1,
                      amp: float = 1e-3, mode: int = 1):
    """Uniform density and background flow u_x0 with a transverse wave
    u_y = amp sin(2 pi mode x / nx); arrays [ny][nx]."""
    x = np.arange(nx, dtype=np.float64)
    uy = np.broadcast_to(amp * np.sin(2 * np.pi * mode * x / nx), (ny, nx))
    return (np.full((ny, nx), rho0), np.full((ny, nx), ux0), np.ascontiguousarray(uy))


def random_fields(nx: int, ny: int, seed: int, rho0: float = 1.0, ux0: float = 0.0,
                  uy0: float = 0.0, drho: float = 0.01, du: float = 0.01):
    """Smooth-free random local equilibria around (rho0, u0) for parity tests."""
    r = np.random.default_rng(seed)
    rho = rho0 + drho * r.standard_normal((ny, nx))
    ux = ux0 + du * r.standard_normal((ny, nx))
    uy = uy0 + du * r.standard_normal((ny, nx))
    return rho, ux, uy


def ensemble_members(n: int = 64, seed: int = 3, seed0: int = 1000):
    """Replica parameters: u_x0 ~ U[0, 0.2], kT log-uniform in [1e-5, 1e-3],
    Philox seed seed0 + r."""
    r = np.random.default_rng(seed)
    ux = r.uniform(0.0, 0.2, n)
    kT = np.exp(r.uniform(math.log(1e-5), math.log(1e-3), n))
    return [{"ux0": float(ux[i]), "kT": float(kT[i]), "seed": seed0 + i} for i in range(n)]


def serving_requests(n: int, rate: float = 50.0, seed: int = 4, side=(64, 2048),
                     steps=(1_000, 100_000), kT=(1e-5, 1e-3), ux=(0.0, 0.2)):
    """Poisson arrivals at `rate` per second; side and step count log-uniform,
    temperature log-uniform, u_x0 uniform; request seed = request index."""
    r = np.random.default_rng(seed)
    gaps = r.exponential(1.0 / rate, n)
    t = np.cumsum(gaps)
    sides = np.rint(np.exp(r.uniform(math.log(side[0]), math.log(side[1]), n))).astype(int)
    nst = np.rint(np.exp(r.uniform(math.log(steps[0]), math.log(steps[1]), n))).astype(int)
    kts = np.exp(r.uniform(math.log(kT[0]), math.log(kT[1]), n))
    uxs = r.uniform(ux[0], ux[1], n)
    return [{"t": float(t[i]), "side": int(sides[i]), "nsteps": int(nst[i]),
             "kT": float(kts[i]), "ux0": float(uxs[i]), "seed": i} for i in range(n)]
