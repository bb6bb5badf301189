"""ctypes wrapper of the D3Q19 oracle (``flbref3.c``; test infrastructure
only, like the rest of this package).  The model, its basis and its noise
draw are described in ``flbref3.h``."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import OracleError, _check, _dp, lib as _lib

BASIS_FNORM_LOCAL, BASIS_HERMITE = 0, 1
Q = 19


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("basis", C.c_int32),
        ("rho0", C.c_double), ("ux0", C.c_double), ("uy0", C.c_double), ("uz0", C.c_double),
        ("kT", C.c_double), ("tau", C.c_double * 15), ("seed", C.c_uint64),
        ("sample_every", C.c_int32), ("block_steps", C.c_int32),
    ]


class Cov(C.Structure):
    _fields_ = [("nsamples", C.c_uint64), ("nblocks", C.c_uint64),
                ("mean_df", C.c_double * 19), ("cov_f", C.c_double * 361),
                ("se_cov_f", C.c_double * 361)]


_ready = False


def lib():
    global _ready
    L = _lib()
    if not _ready:
        d = C.POINTER(C.c_double)
        i32 = C.POINTER(C.c_int32)
        L.flbref3_velocities.argtypes = [i32, i32, i32, d]
        L.flbref3_basis.argtypes = [d]
        L.flbref3_equilibrium.restype = C.c_double
        L.flbref3_equilibrium.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double,
                                          C.c_double]
        L.flbref3_fnorm_basis.argtypes = [C.c_double, C.c_double, C.c_double, d]
        L.flbref3_site_gaussians.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, d]
        L.flbref3_collide.argtypes = [C.POINTER(Params), d, C.c_uint64, C.c_uint64, d]
        L.flbref3_lattice_create.argtypes = [C.POINTER(Params), C.POINTER(C.c_void_p)]
        L.flbref3_lattice_set_populations.argtypes = [C.c_void_p, d, C.c_uint64]
        L.flbref3_lattice_step.argtypes = [C.c_void_p, C.c_uint64]
        L.flbref3_lattice_read_populations.argtypes = [C.c_void_p, d]
        L.flbref3_lattice_read_covariance.argtypes = [C.c_void_p, C.POINTER(Cov)]
        L.flbref3_lattice_reset_stats.argtypes = [C.c_void_p]
        L.flbref3_lattice_time.argtypes = [C.c_void_p]
        L.flbref3_lattice_time.restype = C.c_uint64
        L.flbref3_lattice_destroy.argtypes = [C.c_void_p]
        _ready = True
    return L


def velocities():
    vx, vy, vz = (np.zeros(Q, np.int32) for _ in range(3))
    w = np.zeros(Q)
    lib().flbref3_velocities(vx.ctypes.data_as(C.POINTER(C.c_int32)),
                             vy.ctypes.data_as(C.POINTER(C.c_int32)),
                             vz.ctypes.data_as(C.POINTER(C.c_int32)), _dp(w))
    return vx, vy, vz, w


def basis() -> np.ndarray:
    m = np.zeros((Q, Q))
    lib().flbref3_basis(_dp(m))
    return m


def equilibrium(rho, ux, uy, uz) -> np.ndarray:
    return np.array([lib().flbref3_equilibrium(i, rho, ux, uy, uz) for i in range(Q)])


def fnorm_basis(ux, uy, uz) -> np.ndarray:
    m = np.zeros((Q, Q))
    _check(lib().flbref3_fnorm_basis(ux, uy, uz, _dp(m)), "fnorm_basis3")
    return m


def site_gaussians(seed, site, step, tag=0) -> np.ndarray:
    n = np.zeros(15)
    lib().flbref3_site_gaussians(seed, site, step, tag, _dp(n))
    return n


def make_params(nx, ny, nz, rho0=1.0, ux0=0.0, uy0=0.0, uz0=0.0, kT=0.0, tau=(1.0,) * 15,
                seed=1, basis=BASIS_FNORM_LOCAL, sample_every=0, block_steps=0) -> Params:
    tau = tuple(tau)
    if len(tau) == 1:
        tau = tau * 15
    return Params(nx, ny, nz, basis, rho0, ux0, uy0, uz0, kT, (C.c_double * 15)(*tau), seed,
                  sample_every, block_steps)


def collide(p: Params, f, site=0, step=0) -> np.ndarray:
    fi = np.ascontiguousarray(f, dtype=float)
    fo = np.zeros(Q)
    _check(lib().flbref3_collide(C.byref(p), _dp(fi), site, step, _dp(fo)), "collide3")
    return fo


class Lattice:
    def __init__(self, p: Params):
        self.p = p
        h = C.c_void_p()
        _check(lib().flbref3_lattice_create(C.byref(p), C.byref(h)), "lattice3_create")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None):
            lib().flbref3_lattice_destroy(self.h)
            self.h = None

    def set_populations(self, f, t=0):
        fa = np.ascontiguousarray(f, dtype=float)
        _check(lib().flbref3_lattice_set_populations(self.h, _dp(fa), t), "set_populations3")

    def step(self, n: int):
        _check(lib().flbref3_lattice_step(self.h, n), "step3")

    @property
    def t(self) -> int:
        return int(lib().flbref3_lattice_time(self.h))

    def populations(self) -> np.ndarray:
        f = np.zeros((Q, self.p.nz, self.p.ny, self.p.nx))
        _check(lib().flbref3_lattice_read_populations(self.h, _dp(f)), "read3")
        return f

    def covariance(self) -> dict:
        c = Cov()
        _check(lib().flbref3_lattice_read_covariance(self.h, C.byref(c)), "cov3")
        return {"nsamples": int(c.nsamples), "nblocks": int(c.nblocks),
                "mean_df": np.array(c.mean_df[:]),
                "cov_f": np.array(c.cov_f[:]).reshape(Q, Q),
                "se_cov_f": np.array(c.se_cov_f[:]).reshape(Q, Q)}

    def reset_stats(self):
        _check(lib().flbref3_lattice_reset_stats(self.h), "reset3")
