"""FP64 CPU oracle for the fluctuating D2Q9 step (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does.

The numerics live in ``flbref.c`` (plain C, FP64, ``-ffp-contract=off``);
this module builds it with gcc and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libflbref.so")
_SRC = os.path.join(_HERE, "flbref.c")

OK = 0
E_ARG = -1
E_OOM = -2
E_INVALID_VELOCITY = -4
E_NONFINITE = -5

BASIS_FNORM_LOCAL, BASIS_HERMITE, BASIS_FNORM_LUT = 0, 1, 2
INIT_EQUILIBRIUM, INIT_THERMAL, INIT_FIELDS = 0, 1, 2
AT_LOCAL, AT_U0, AT_HERMITE = 0, 1, 2


_SRC3 = os.path.join(_HERE, "flbref3.c")


def build(force: bool = False) -> str:
    """Compile ``libflbref.so`` (D2Q9 and D3Q19 oracles) with gcc (always when
    ``force``)."""
    deps = [_SRC, _SRC3] + [os.path.join(_HERE, h) for h in ("flbref.h", "flbref3.h")]
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < max(
        os.path.getmtime(f) for f in deps
    ):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-Wall", "-fopenmp", "-fPIC",
             "-shared", "-o", tmp, _SRC, _SRC3, "-lm"]
        )
        os.replace(tmp, _SO)
    return _SO


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("rho0", C.c_double), ("ux0", C.c_double), ("uy0", C.c_double),
        ("kT", C.c_double), ("tau", C.c_double * 6), ("seed", C.c_uint64),
        ("precision", C.c_int32), ("basis", C.c_int32), ("init", C.c_int32),
        ("sample_every", C.c_int32), ("sk_every", C.c_int32), ("block_steps", C.c_int32),
    ]


class Cov(C.Structure):
    _fields_ = [
        ("nsamples", C.c_uint64), ("nblocks", C.c_uint64),
        ("mean_df", C.c_double * 9), ("cov_f", C.c_double * 81),
        ("cov_m_fnorm_u0", C.c_double * 81), ("cov_m_hermite", C.c_double * 81),
        ("se_cov_f", C.c_double * 81), ("se_cov_m", C.c_double * 81),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d = C.POINTER(C.c_double)
        L = _lib
        L.flbref_equilibrium.restype = C.c_double
        L.flbref_equilibrium.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double]
        L.flbref_fnorm_basis.argtypes = [C.c_double, C.c_double, d]
        L.flbref_lut_basis.argtypes = [C.c_double, C.c_double, d, d]
        L.flbref_hermite_matrix.argtypes = [d]
        L.flbref_velocities.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_int32), d]
        L.flbref_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                           C.POINTER(C.c_uint32)]
        L.flbref_site_gaussians.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, d]
        L.flbref_collide.argtypes = [C.POINTER(Params), d, C.c_uint64, C.c_uint64, d]
        L.flbref_collide_lut_at.argtypes = [C.POINTER(Params), d, C.c_uint64, C.c_uint64,
                                            C.c_int32, C.c_int32, d]
        L.flbref_set_threads.argtypes = [C.c_int]
        L.flbref_lattice_create.argtypes = [C.POINTER(Params), C.POINTER(C.c_void_p)]
        L.flbref_lattice_set_fields.argtypes = [C.c_void_p, d, d, d]
        L.flbref_lattice_set_populations.argtypes = [C.c_void_p, d, C.c_uint64]
        L.flbref_lattice_step.argtypes = [C.c_void_p, C.c_uint64]
        L.flbref_lattice_read_populations.argtypes = [C.c_void_p, d]
        L.flbref_lattice_read_moments.argtypes = [C.c_void_p, C.c_int32, d]
        L.flbref_lattice_read_covariance.argtypes = [C.c_void_p, C.POINTER(Cov)]
        L.flbref_lattice_read_structure_factor.argtypes = [C.c_void_p, C.c_int32, d]
        L.flbref_lattice_read_fourier_mode.argtypes = [C.c_void_p, C.c_int32, C.c_int32,
                                                       C.c_int32, d]
        L.flbref_lattice_reset_stats.argtypes = [C.c_void_p]
        L.flbref_lattice_time.argtypes = [C.c_void_p]
        L.flbref_lattice_time.restype = C.c_uint64
        L.flbref_lattice_error_step.argtypes = [C.c_void_p]
        L.flbref_lattice_error_step.restype = C.c_int64
        L.flbref_lattice_destroy.argtypes = [C.c_void_p]
    return _lib


def set_threads(n: int):
    """Threads of the lattice calls' per-site loops (results do not depend
    on it)."""
    lib().flbref_set_threads(int(n))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle error {code}")
        self.code = code


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


# ---------------------------------------------------------------- site level
def velocities():
    vx = (C.c_int32 * 9)()
    vy = (C.c_int32 * 9)()
    w = np.zeros(9)
    lib().flbref_velocities(vx, vy, _dp(w))
    return np.array(vx[:]), np.array(vy[:]), w


def hermite_matrix() -> np.ndarray:
    m = np.zeros(81)
    lib().flbref_hermite_matrix(_dp(m))
    return m.reshape(9, 9)


def equilibrium(rho: float, ux: float, uy: float) -> np.ndarray:
    return np.array([lib().flbref_equilibrium(i, rho, ux, uy) for i in range(9)])


def fnorm_basis(ux: float, uy: float) -> np.ndarray:
    m = np.zeros(81)
    _check(lib().flbref_fnorm_basis(ux, uy, _dp(m)), "fnorm_basis")
    return m.reshape(9, 9)


def lut_basis(ux: float, uy: float):
    m = np.zeros(81)
    ug = np.zeros(2)
    _check(lib().flbref_lut_basis(ux, uy, _dp(m), _dp(ug)), "lut_basis")
    return m.reshape(9, 9), ug


def philox(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().flbref_philox4x32_10(c, k, o)
    return np.array(o[:], dtype=np.uint32)


def site_gaussians(seed: int, site: int, step: int, tag: int = 0) -> np.ndarray:
    n = np.zeros(6)
    lib().flbref_site_gaussians(seed, site, step, tag, _dp(n))
    return n


def make_params(nx, ny, rho0=1.0, ux0=0.0, uy0=0.0, kT=0.0, tau=(1.0,) * 6, seed=1,
                basis=BASIS_FNORM_LOCAL, init=INIT_EQUILIBRIUM, sample_every=0, sk_every=0,
                block_steps=0, precision=0) -> Params:
    p = Params()
    p.nx, p.ny = int(nx), int(ny)
    p.rho0, p.ux0, p.uy0, p.kT = float(rho0), float(ux0), float(uy0), float(kT)
    for a in range(6):
        p.tau[a] = float(tau[a])
    p.seed = int(seed)
    p.precision, p.basis, p.init = int(precision), int(basis), int(init)
    p.sample_every, p.sk_every, p.block_steps = int(sample_every), int(sk_every), int(block_steps)
    return p


def collide(p: Params, f, site: int = 0, step: int = 0) -> np.ndarray:
    fi = np.ascontiguousarray(f, dtype=np.float64)
    fo = np.zeros(9)
    _check(lib().flbref_collide(C.byref(p), _dp(fi), site, step, _dp(fo)), "collide")
    return fo


def collide_lut_at(p: Params, f, ix: int, iy: int, site: int = 0, step: int = 0) -> np.ndarray:
    """Table-basis collision with the basis at grid point (ix, iy) * 0.02."""
    fi = np.ascontiguousarray(f, dtype=np.float64)
    fo = np.zeros(9)
    _check(lib().flbref_collide_lut_at(C.byref(p), _dp(fi), site, step, ix, iy, _dp(fo)),
           "collide_lut_at")
    return fo


# ------------------------------------------------------------------- lattice
def sk_fields(f: np.ndarray, rho0: float, ux0: float, uy0: float):
    """The fields whose transforms the structure factors average (eqs. (24)-(26),
    measured in the f-norm at (rho0, u0) as in the captions of Figs. 19-21):
    d rho = sum_i f_i - rho0 and dM~^a = sum_i m~^a_i(u0) f_i (a = 1, 2) with
    m~^1 = sqrt3 (v_x - u_x0), m~^2 = sqrt3 (v_y - u_y0), whose value at the
    reference state is zero.  f: populations [9][ny][nx]."""
    vx, vy, _ = velocities()
    s3 = np.sqrt(3.0)
    drho = f.sum(axis=0) - rho0
    m1 = np.tensordot(s3 * (vx - ux0), f, axes=(0, 0))
    m2 = np.tensordot(s3 * (vy - uy0), f, axes=(0, 0))
    return drho, m1, m2


def fourier_coefficient(a: np.ndarray, kx: int, ky: int) -> complex:
    """A(k) = sum_x a(x) exp(-2 pi i (kx x / nx + ky y / ny)) of a field
    a[ny][nx], by its definition (the separable sum)."""
    ny, nx = a.shape
    ex = np.exp(-2j * np.pi * ((kx * np.arange(nx)) % nx) / nx)
    ey = np.exp(-2j * np.pi * ((ky * np.arange(ny)) % ny) / ny)
    return complex(ey @ (a @ ex))


class Lattice:
    """Host FP64 lattice mirroring the GPU library's lattice calls."""

    def __init__(self, p: Params):
        self.p = p
        self.n = p.nx * p.ny
        h = C.c_void_p()
        _check(lib().flbref_lattice_create(C.byref(p), C.byref(h)), "lattice_create")
        self.h = h

    def close(self):
        if self.h:
            lib().flbref_lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fields(self, rho, ux, uy):
        r, a, b = (np.ascontiguousarray(x, dtype=np.float64).ravel() for x in (rho, ux, uy))
        _check(lib().flbref_lattice_set_fields(self.h, _dp(r), _dp(a), _dp(b)), "set_fields")

    def set_populations(self, f, t: int = 0):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, -1)
        _check(lib().flbref_lattice_set_populations(self.h, _dp(f), t), "set_populations")

    def step(self, n: int):
        _check(lib().flbref_lattice_step(self.h, n), "step")

    @property
    def t(self) -> int:
        return int(lib().flbref_lattice_time(self.h))

    @property
    def error_step(self) -> int:
        return int(lib().flbref_lattice_error_step(self.h))

    def populations(self) -> np.ndarray:
        f = np.zeros((9, self.p.ny, self.p.nx))
        _check(lib().flbref_lattice_read_populations(self.h, _dp(f)), "read_populations")
        return f

    def moments(self, at: int = AT_U0) -> np.ndarray:
        m = np.zeros((9, self.p.ny, self.p.nx))
        _check(lib().flbref_lattice_read_moments(self.h, at, _dp(m)), "read_moments")
        return m

    def covariance(self) -> dict:
        c = Cov()
        _check(lib().flbref_lattice_read_covariance(self.h, C.byref(c)), "read_covariance")
        out = {"nsamples": int(c.nsamples), "nblocks": int(c.nblocks),
               "mean_df": np.array(c.mean_df[:])}
        for k in ("cov_f", "cov_m_fnorm_u0", "cov_m_hermite", "se_cov_f", "se_cov_m"):
            out[k] = np.array(getattr(c, k)[:]).reshape(9, 9)
        return out

    def structure_factor(self, which: int) -> np.ndarray:
        o = np.zeros((self.p.ny, self.p.nx))
        _check(lib().flbref_lattice_read_structure_factor(self.h, which, _dp(o)), "read_sk")
        return o

    def fourier_mode(self, which: int, kx: int, ky: int) -> complex:
        o = np.zeros(2)
        _check(lib().flbref_lattice_read_fourier_mode(self.h, which, kx, ky, _dp(o)), "mode")
        return complex(o[0], o[1])

    def reset_stats(self):
        _check(lib().flbref_lattice_reset_stats(self.h), "reset_stats")
