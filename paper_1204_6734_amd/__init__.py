"""Python binding of libflb (fluctuating D2Q9 lattice Boltzmann, f-norm basis).

Argument marshalling only: every step of the method runs in the HIP kernels
of ``libflb.so`` (built in-tree by ``paper_1204_6734_amd.build``).  Importing
this package does not load the library; the first use does, and fails loudly
if it is missing.

Method: Kaehler & Wagner, "A fluctuating lattice-Boltzmann method with
improved Galilean invariance" (collision eq. (6), noise eq. (20), f-norm
basis Sec. IV, correlators eqs. (16)/(23), structure factors eqs. (24)-(26)).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libflb.so")

OK = 0
E_ARG, E_OOM, E_HIP, E_INVALID_VELOCITY, E_NONFINITE, E_ADMISSION, E_STATE = (
    -1, -2, -3, -4, -5, -6, -7)
FP64, FP32_SHIFTED = 0, 1
BASIS_FNORM_LOCAL, BASIS_HERMITE, BASIS_FNORM_LUT = 0, 1, 2
INIT_EQUILIBRIUM, INIT_THERMAL, INIT_FIELDS = 0, 1, 2
AT_LOCAL, AT_U0, AT_HERMITE = 0, 1, 2
SK_RHO, SK_JX, SK_JY, SK_JXJY_RE, SK_JXJY_IM = 0, 1, 2, 3, 4


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
        ("se_cov_m_hermite", C.c_double * 81),
    ]


class ServerConfig(C.Structure):
    _fields_ = [
        ("mem_budget_bytes", C.c_size_t), ("max_slots", C.c_int32),
        ("chunk_steps", C.c_int32), ("precision", C.c_int32), ("basis", C.c_int32),
        ("threaded", C.c_int32),
    ]


class Request(C.Structure):
    _fields_ = [("p", Params), ("nsteps", C.c_uint64), ("tag", C.c_uint64)]


class Result(C.Structure):
    _fields_ = [
        ("id", C.c_uint64), ("tag", C.c_uint64), ("status", C.c_int32), ("pad_", C.c_int32),
        ("nsteps", C.c_uint64), ("t_submit", C.c_double), ("t_admit", C.c_double),
        ("t_done", C.c_double), ("cov", Cov),
    ]


class LaunchConfig(C.Structure):
    _fields_ = [("tiles_per_block", C.c_int32), ("grid_blocks", C.c_int32),
                ("ms_per_step", C.c_double)]


class Params3(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("precision", C.c_int32),
        ("basis", C.c_int32), ("sample_every", C.c_int32), ("block_steps", C.c_int32),
        ("pad_", C.c_int32), ("rho0", C.c_double), ("ux0", C.c_double), ("uy0", C.c_double),
        ("uz0", C.c_double), ("kT", C.c_double), ("tau", C.c_double * 15),
        ("seed", C.c_uint64),
    ]


class Cov3(C.Structure):
    _fields_ = [("nsamples", C.c_uint64), ("nblocks", C.c_uint64),
                ("mean_df", C.c_double * 19), ("cov_f", C.c_double * 361),
                ("se_cov_f", C.c_double * 361)]


class FlbError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what} failed ({code}): {msg}")
        self.code = code


_lib = None

_SIGS = {
    "flb_lattice_create": [C.POINTER(Params), C.c_void_p, C.POINTER(C.c_void_p)],
    "flb_lattice_create_on": [C.POINTER(Params), C.c_void_p, C.c_size_t, C.c_void_p,
                              C.POINTER(C.c_void_p)],
    "flb_lattice_set_fields": [C.c_void_p] + [C.POINTER(C.c_double)] * 3,
    "flb_lattice_set_populations": [C.c_void_p, C.POINTER(C.c_double), C.c_uint64],
    "flb_lattice_step": [C.c_void_p, C.c_uint64],
    "flb_lattice_set_graph_chunk": [C.c_void_p, C.c_int32],
    "flb_lattice_sync": [C.c_void_p],
    "flb_lattice_read_populations": [C.c_void_p, C.POINTER(C.c_double)],
    "flb_lattice_read_rows": [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double)],
    "flb_lattice_read_moments": [C.c_void_p, C.c_int32, C.POINTER(C.c_double)],
    "flb_lattice_read_covariance": [C.c_void_p, C.POINTER(Cov)],
    "flb_lattice_read_structure_factor": [C.c_void_p, C.c_int32, C.POINTER(C.c_double)],
    "flb_lattice_read_fourier_mode": [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                      C.POINTER(C.c_double)],
    "flb_lattice_reset_stats": [C.c_void_p],
    "flb_lattice_checkpoint": [C.c_void_p, C.c_void_p, C.c_size_t],
    "flb_lattice_restore": [C.c_void_p, C.c_void_p, C.c_size_t],
    "flb_lattice_profile": [C.c_void_p, C.c_int32],
    "flb_lattice_kernel_time": [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)],
    "flb_ensemble_create": [C.POINTER(Params), C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)],
    "flb_ensemble_set_graph_chunk": [C.c_void_p, C.c_int32],
    "flb_ensemble_step": [C.c_void_p, C.c_uint64],
    "flb_ensemble_sync": [C.c_void_p],
    "flb_ensemble_read_populations": [C.c_void_p, C.c_int32, C.POINTER(C.c_double)],
    "flb_ensemble_read_covariance": [C.c_void_p, C.c_int32, C.POINTER(Cov)],
    "flb_ensemble_reset_stats": [C.c_void_p],
    "flb_ensemble_profile": [C.c_void_p, C.c_int32],
    "flb_ensemble_kernel_time": [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)],
    "flb_lattice_autotune": [C.c_void_p, C.c_int32, C.POINTER(LaunchConfig), C.c_int32,
                             C.POINTER(C.c_int32)],
    "flb_ensemble_autotune": [C.c_void_p, C.c_int32, C.POINTER(LaunchConfig), C.c_int32,
                              C.POINTER(C.c_int32)],
    "flb_lattice_set_launch": [C.c_void_p, C.POINTER(LaunchConfig)],
    "flb_ensemble_set_launch": [C.c_void_p, C.POINTER(LaunchConfig)],
    "flb_lattice_get_launch": [C.c_void_p, C.POINTER(LaunchConfig)],
    "flb_ensemble_get_launch": [C.c_void_p, C.POINTER(LaunchConfig)],
    "flb3_lattice_create": [C.POINTER(Params3), C.c_void_p, C.POINTER(C.c_void_p)],
    "flb3_lattice_set_populations": [C.c_void_p, C.POINTER(C.c_double), C.c_uint64],
    "flb3_lattice_step": [C.c_void_p, C.c_uint64],
    "flb3_lattice_sync": [C.c_void_p],
    "flb3_lattice_read_populations": [C.c_void_p, C.POINTER(C.c_double)],
    "flb3_lattice_read_covariance": [C.c_void_p, C.POINTER(Cov3)],
    "flb3_lattice_reset_stats": [C.c_void_p],
    "flb3_lattice_profile": [C.c_void_p, C.c_int32],
    "flb3_lattice_kernel_time": [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)],
    "flb_copy_probe": [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double)],
    "flb_stream_copy_probe": [C.c_uint64, C.c_int32, C.POINTER(C.c_double)],
    "flb_step_noalloc": [C.POINTER(Params), C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p,
                         C.c_void_p, C.c_void_p],
    "flb_lattice_population_buffer": [C.c_void_p, C.POINTER(C.c_void_p),
                                      C.POINTER(C.c_size_t), C.POINTER(C.c_uint64)],
    "flb_server_create": [C.POINTER(ServerConfig), C.c_void_p, C.POINTER(C.c_void_p)],
    "flb_server_submit": [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)],
    "flb_server_pump": [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)],
    "flb_server_poll": [C.c_void_p, C.POINTER(Result), C.c_int32, C.POINTER(C.c_int32)],
    "flb_server_drain": [C.c_void_p],
    "flb_server_stats": [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                         C.POINTER(C.c_uint64), C.POINTER(C.c_double), C.POINTER(C.c_double)],
}
_VOID = {"flb_lattice_destroy": [C.c_void_p], "flb_ensemble_destroy": [C.c_void_p],
         "flb_server_destroy": [C.c_void_p], "flb3_lattice_destroy": [C.c_void_p]}


def load(path: str | None = None):
    """Load libflb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # One HIP runtime per process: PyTorch ships its own copy of the HIP
    # runtime under the same soname; loading torch first makes libflb bind
    # to that copy, so torch tensors and streams and libflb share a runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"libflb.so not found at {p}: run python -m paper_1204_6734_amd.build")
    lib = C.CDLL(p)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    for name, args in _VOID.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = None
    lib.flb_last_error.restype = C.c_char_p
    lib.flb_lattice_bytes.argtypes = [C.POINTER(Params)]
    lib.flb_lattice_bytes.restype = C.c_size_t
    lib.flb_population_bytes.argtypes = [C.POINTER(Params)]
    lib.flb_population_bytes.restype = C.c_size_t
    lib.flb_lattice_checkpoint_bytes.argtypes = [C.c_void_p]
    lib.flb_lattice_checkpoint_bytes.restype = C.c_size_t
    lib.flb_server_request_bytes.argtypes = [C.POINTER(ServerConfig), C.POINTER(Request)]
    lib.flb_server_request_bytes.restype = C.c_size_t
    lib.flb3_lattice_error_step.argtypes = [C.c_void_p]
    lib.flb3_lattice_error_step.restype = C.c_int64
    for name in ("flb_lattice_time", "flb_ensemble_time", "flb3_lattice_time"):
        getattr(lib, name).argtypes = [C.c_void_p]
        getattr(lib, name).restype = C.c_uint64
    lib.flb_lattice_error_step.argtypes = [C.c_void_p]
    lib.flb_lattice_error_step.restype = C.c_int64
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc != OK:
        raise FlbError(rc, what, load().flb_last_error().decode(errors="replace"))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _host_f64(x, size: int, what: str) -> np.ndarray:
    """Contiguous FP64 copy (or view) of x, which must hold `size` values: the
    library reads exactly that many from the pointer it is given."""
    a = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    if a.size != size:
        raise ValueError(f"{what}: expected {size} values, got {a.size}")
    return a


def make_params(nx, ny, rho0=1.0, ux0=0.0, uy0=0.0, kT=0.0, tau=(1.0,) * 6, seed=1,
                precision=FP32_SHIFTED, basis=BASIS_FNORM_LOCAL, init=INIT_EQUILIBRIUM,
                sample_every=0, sk_every=0, block_steps=0) -> Params:
    p = Params()
    p.nx, p.ny = int(nx), int(ny)
    p.rho0, p.ux0, p.uy0, p.kT = float(rho0), float(ux0), float(uy0), float(kT)
    for a in range(6):
        p.tau[a] = float(tau[a])
    p.seed = int(seed)
    p.precision, p.basis, p.init = int(precision), int(basis), int(init)
    p.sample_every, p.sk_every, p.block_steps = int(sample_every), int(sk_every), int(block_steps)
    return p


def _cov_dict(c: Cov) -> dict:
    out = {"nsamples": int(c.nsamples), "nblocks": int(c.nblocks),
           "mean_df": np.array(c.mean_df[:])}
    for k in ("cov_f", "cov_m_fnorm_u0", "cov_m_hermite", "se_cov_f", "se_cov_m",
              "se_cov_m_hermite"):
        out[k] = np.array(getattr(c, k)[:]).reshape(9, 9)
    return out


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(getattr(stream, "cuda_stream", stream))


class _Tunable:
    """Launch-shape control shared by lattices and ensembles (flb_*_autotune,
    flb_*_set_launch, flb_*_get_launch)."""

    _kind = ""

    def autotune(self, reps: int = 5, max_results: int = 32) -> list:
        """Time every launch shape on a copy of the state and keep the fastest;
        returns the measurements, fastest first, as dicts."""
        out = (LaunchConfig * max_results)()
        n = C.c_int32()
        fn = getattr(load(), f"flb_{self._kind}_autotune")
        _check(fn(self.h, reps, out, max_results, C.byref(n)), "autotune")
        return [{"tiles_per_block": c.tiles_per_block, "grid_blocks": c.grid_blocks,
                 "ms_per_step": c.ms_per_step} for c in out[:min(n.value, max_results)]]

    def set_launch(self, tiles_per_block: int = 1, grid_blocks: int = 0):
        c = LaunchConfig(tiles_per_block, grid_blocks, 0.0)
        _check(getattr(load(), f"flb_{self._kind}_set_launch")(self.h, C.byref(c)), "set_launch")

    def get_launch(self) -> dict:
        c = LaunchConfig()
        _check(getattr(load(), f"flb_{self._kind}_get_launch")(self.h, C.byref(c)), "get_launch")
        return {"tiles_per_block": c.tiles_per_block, "grid_blocks": c.grid_blocks}


class Lattice(_Tunable):
    """One periodic lattice on the GPU (flb_lattice_*)."""

    _kind = "lattice"

    def __init__(self, p: Params, stream=None, device_buffer=None):
        lib = load()
        self.p = p
        self.n = p.nx * p.ny
        h = C.c_void_p()
        if device_buffer is not None:
            ptr, nbytes = device_buffer
            _check(lib.flb_lattice_create_on(C.byref(p), C.c_void_p(ptr), nbytes,
                                             _stream_ptr(stream), C.byref(h)), "lattice_create_on")
        else:
            _check(lib.flb_lattice_create(C.byref(p), _stream_ptr(stream), C.byref(h)),
                   "lattice_create")
        self.h = h

    @staticmethod
    def bytes_needed(p: Params) -> int:
        return int(load().flb_lattice_bytes(C.byref(p)))

    def population_buffer(self):
        """(device address, bytes, time) of the lattice's population storage
        (flb_lattice_population_buffer)."""
        ptr, nbytes, t = C.c_void_p(), C.c_size_t(), C.c_uint64()
        _check(load().flb_lattice_population_buffer(self.h, C.byref(ptr), C.byref(nbytes),
                                                    C.byref(t)), "population_buffer")
        return int(ptr.value or 0), int(nbytes.value), int(t.value)

    def close(self):
        if getattr(self, "h", None):
            load().flb_lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_fields(self, rho, ux, uy):
        r, a, b = (_host_f64(x, self.n, "set_fields") for x in (rho, ux, uy))
        _check(load().flb_lattice_set_fields(self.h, _dp(r), _dp(a), _dp(b)), "set_fields")

    def set_populations(self, f, t: int = 0):
        f = _host_f64(f, 9 * self.n, "set_populations")
        _check(load().flb_lattice_set_populations(self.h, _dp(f), t), "set_populations")

    def step(self, n: int):
        _check(load().flb_lattice_step(self.h, n), "step")

    def set_graph_chunk(self, steps: int):
        """Replay captured hipGraphs of `steps` steps (0: launch eagerly);
        results are unchanged (flb_lattice_set_graph_chunk)."""
        _check(load().flb_lattice_set_graph_chunk(self.h, steps), "set_graph_chunk")

    def sync(self):
        _check(load().flb_lattice_sync(self.h), "sync")

    @property
    def t(self) -> int:
        return int(load().flb_lattice_time(self.h))

    @property
    def error_step(self) -> int:
        return int(load().flb_lattice_error_step(self.h))

    def populations(self) -> np.ndarray:
        f = np.empty((9, self.p.ny, self.p.nx))
        _check(load().flb_lattice_read_populations(self.h, _dp(f)), "read_populations")
        return f

    def rows(self, y0: int, nrows: int) -> np.ndarray:
        """Populations of rows [y0, y0 + nrows), [9][nrows][nx]."""
        f = np.empty((9, nrows, self.p.nx))
        _check(load().flb_lattice_read_rows(self.h, y0, nrows, _dp(f)), "read_rows")
        return f

    def moments(self, at: int = AT_U0) -> np.ndarray:
        m = np.empty((9, self.p.ny, self.p.nx))
        _check(load().flb_lattice_read_moments(self.h, at, _dp(m)), "read_moments")
        return m

    def covariance(self) -> dict:
        c = Cov()
        _check(load().flb_lattice_read_covariance(self.h, C.byref(c)), "read_covariance")
        return _cov_dict(c)

    def structure_factor(self, which: int) -> np.ndarray:
        o = np.empty((self.p.ny, self.p.nx))
        _check(load().flb_lattice_read_structure_factor(self.h, which, _dp(o)), "read_sk")
        return o

    def fourier_mode(self, which: int, kx: int, ky: int) -> complex:
        o = np.empty(2)
        _check(load().flb_lattice_read_fourier_mode(self.h, which, kx, ky, _dp(o)), "mode")
        return complex(o[0], o[1])

    def reset_stats(self):
        _check(load().flb_lattice_reset_stats(self.h), "reset_stats")

    def checkpoint(self) -> bytes:
        n = int(load().flb_lattice_checkpoint_bytes(self.h))
        buf = C.create_string_buffer(n)
        _check(load().flb_lattice_checkpoint(self.h, buf, n), "checkpoint")
        return buf.raw

    def restore(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        _check(load().flb_lattice_restore(self.h, buf, len(blob)), "restore")

    def profile(self, on: bool = True):
        _check(load().flb_lattice_profile(self.h, 1 if on else 0), "profile")

    def kernel_time(self):
        ms = C.c_double()
        n = C.c_uint64()
        _check(load().flb_lattice_kernel_time(self.h, C.byref(ms), C.byref(n)), "kernel_time")
        return ms.value, n.value


class Ensemble(_Tunable):
    """Replicas of one lattice shape in one batched launch (flb_ensemble_*)."""

    _kind = "ensemble"

    def __init__(self, params: list, stream=None, graph_chunk: int = 0):
        lib = load()
        self.params = list(params)
        arr = (Params * len(self.params))(*self.params)
        h = C.c_void_p()
        _check(lib.flb_ensemble_create(arr, len(self.params), _stream_ptr(stream), C.byref(h)),
               "ensemble_create")
        self.h = h
        if graph_chunk:
            _check(lib.flb_ensemble_set_graph_chunk(self.h, graph_chunk), "set_graph_chunk")

    def close(self):
        if getattr(self, "h", None):
            load().flb_ensemble_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int):
        _check(load().flb_ensemble_step(self.h, n), "ensemble_step")

    def sync(self):
        _check(load().flb_ensemble_sync(self.h), "ensemble_sync")

    @property
    def t(self) -> int:
        return int(load().flb_ensemble_time(self.h))

    def populations(self, i: int) -> np.ndarray:
        p = self.params[i]
        f = np.empty((9, p.ny, p.nx))
        _check(load().flb_ensemble_read_populations(self.h, i, _dp(f)), "ensemble_read")
        return f

    def covariance(self, i: int) -> dict:
        c = Cov()
        _check(load().flb_ensemble_read_covariance(self.h, i, C.byref(c)), "ensemble_cov")
        return _cov_dict(c)

    def reset_stats(self):
        _check(load().flb_ensemble_reset_stats(self.h), "ensemble_reset_stats")

    def profile(self, on: bool = True):
        _check(load().flb_ensemble_profile(self.h, 1 if on else 0), "profile")

    def kernel_time(self):
        ms = C.c_double()
        n = C.c_uint64()
        _check(load().flb_ensemble_kernel_time(self.h, C.byref(ms), C.byref(n)), "kernel_time")
        return ms.value, n.value


def population_bytes(p: Params) -> int:
    """Bytes of a lattice's population storage (flb_population_bytes)."""
    return int(load().flb_population_bytes(C.byref(p)))


def step_noalloc(p: Params, pop_ptr: int, t0: int, nsteps: int, sums_ptr: int = 0,
                 status_ptr: int = 0, stream=None):
    """flb_step_noalloc: nsteps updates of caller-held device populations
    (pop_ptr) from time t0, the correlator sums into the 54 doubles at
    sums_ptr and the outcome code into the int32 at status_ptr (device
    addresses; 0 for none).  Asynchronous on `stream`; allocates nothing."""
    _check(load().flb_step_noalloc(C.byref(p), C.c_void_p(pop_ptr), t0, nsteps,
                                   C.c_void_p(sums_ptr or None), C.c_void_p(status_ptr or None),
                                   _stream_ptr(stream)), "step_noalloc")


def copy_probe(nx: int, ny: int, precision: int = FP32_SHIFTED, reps: int = 20) -> float:
    """Device time (ms) of one pass of the step kernel's memory traffic with no
    arithmetic over an nx x ny lattice (flb_copy_probe): the practical
    ceiling of the step's access pattern."""
    ms = C.c_double()
    _check(load().flb_copy_probe(nx, ny, precision, reps, C.byref(ms)), "copy_probe")
    return ms.value


def stream_copy_probe(nbytes: int, reps: int = 20) -> float:
    """Device time (ms) of one contiguous copy of nbytes, 16 bytes per thread
    (flb_stream_copy_probe): the device's streaming ceiling."""
    ms = C.c_double()
    _check(load().flb_stream_copy_probe(nbytes, reps, C.byref(ms)), "stream_copy_probe")
    return ms.value


def make_params3(nx, ny, nz, rho0=1.0, ux0=0.0, uy0=0.0, uz0=0.0, kT=0.0, tau=(1.0,) * 15,
                 seed=1, precision=FP32_SHIFTED, basis=BASIS_FNORM_LOCAL, sample_every=0,
                 block_steps=0) -> Params3:
    """D3Q19 parameters (flb3_params)."""
    tau = tuple(tau)
    if len(tau) == 1:
        tau = tau * 15
    return Params3(nx, ny, nz, precision, basis, sample_every, block_steps, 0, rho0, ux0, uy0,
                   uz0, kT, (C.c_double * 15)(*tau), seed)


class Lattice3:
    """One periodic D3Q19 lattice on the GPU (flb3_lattice_*)."""

    def __init__(self, p: Params3, stream=None):
        lib = load()
        self.p = p
        h = C.c_void_p()
        _check(lib.flb3_lattice_create(C.byref(p), _stream_ptr(stream), C.byref(h)),
               "lattice3_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().flb3_lattice_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_populations(self, f, t: int = 0):
        fa = _host_f64(f, 19 * self.p.nx * self.p.ny * self.p.nz, "set_populations3")
        _check(load().flb3_lattice_set_populations(self.h, _dp(fa), t), "set_populations3")

    def step(self, n: int):
        _check(load().flb3_lattice_step(self.h, n), "step3")

    def sync(self):
        _check(load().flb3_lattice_sync(self.h), "sync3")

    @property
    def t(self) -> int:
        return int(load().flb3_lattice_time(self.h))

    @property
    def error_step(self) -> int:
        return int(load().flb3_lattice_error_step(self.h))

    def populations(self) -> np.ndarray:
        f = np.empty((19, self.p.nz, self.p.ny, self.p.nx))
        _check(load().flb3_lattice_read_populations(self.h, _dp(f)), "read3")
        return f

    def covariance(self) -> dict:
        c = Cov3()
        _check(load().flb3_lattice_read_covariance(self.h, C.byref(c)), "cov3")
        return {"nsamples": int(c.nsamples), "nblocks": int(c.nblocks),
                "mean_df": np.array(c.mean_df[:]),
                "cov_f": np.array(c.cov_f[:]).reshape(19, 19),
                "se_cov_f": np.array(c.se_cov_f[:]).reshape(19, 19)}

    def reset_stats(self):
        _check(load().flb3_lattice_reset_stats(self.h), "reset3")

    def profile(self, on: bool = True):
        _check(load().flb3_lattice_profile(self.h, 1 if on else 0), "profile3")

    def kernel_time(self):
        ms = C.c_double()
        n = C.c_uint64()
        _check(load().flb3_lattice_kernel_time(self.h, C.byref(ms), C.byref(n)), "kernel_time3")
        return ms.value, n.value


class Server:
    """Continuous-batching simulation server (flb_server_*)."""

    def __init__(self, mem_budget_bytes: int, max_slots: int = 64, chunk_steps: int = 100,
                 precision: int = FP32_SHIFTED, basis: int = BASIS_FNORM_LOCAL,
                 threaded: bool = True, stream=None):
        lib = load()
        cfg = ServerConfig()
        cfg.mem_budget_bytes = int(mem_budget_bytes)
        cfg.max_slots, cfg.chunk_steps = int(max_slots), int(chunk_steps)
        cfg.precision, cfg.basis, cfg.threaded = int(precision), int(basis), 1 if threaded else 0
        h = C.c_void_p()
        _check(lib.flb_server_create(C.byref(cfg), _stream_ptr(stream), C.byref(h)),
               "server_create")
        self.h = h
        self.cfg = cfg

    def close(self):
        if getattr(self, "h", None):
            load().flb_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def request_bytes(p: Params, nsteps: int = 1, precision: int = FP32_SHIFTED,
                      basis: int = BASIS_FNORM_LOCAL) -> int:
        """Device bytes the request occupies in a server storing `precision`
        (the request's own precision field is not used)."""
        cfg = ServerConfig()
        cfg.precision, cfg.basis = precision, basis
        r = Request(p=p, nsteps=nsteps, tag=0)
        return int(load().flb_server_request_bytes(C.byref(cfg), C.byref(r)))

    def submit(self, p: Params, nsteps: int, tag: int = 0) -> int:
        r = Request(p=p, nsteps=int(nsteps), tag=int(tag))
        rid = C.c_uint64()
        _check(load().flb_server_submit(self.h, C.byref(r), C.byref(rid)), "submit")
        return rid.value

    def pump(self, max_chunks: int = 1) -> int:
        did = C.c_int32()
        _check(load().flb_server_pump(self.h, max_chunks, C.byref(did)), "pump")
        return did.value

    def poll(self, max_results: int = 1024) -> list:
        """Completed results, oldest first.  If the server has stopped on an
        error, raises FlbError with the results delivered by this call in its
        `results` attribute."""
        buf = (Result * max_results)()
        n = C.c_int32()
        rc = load().flb_server_poll(self.h, buf, max_results, C.byref(n))
        out = []
        for k in range(n.value):
            r = buf[k]
            out.append({"id": r.id, "tag": r.tag, "status": r.status, "nsteps": r.nsteps,
                        "t_submit": r.t_submit, "t_admit": r.t_admit, "t_done": r.t_done,
                        "cov": _cov_dict(r.cov)})
        try:
            _check(rc, "poll")
        except FlbError as e:
            e.results = out
            raise
        return out

    def drain(self):
        _check(load().flb_server_drain(self.h), "drain")

    def stats(self) -> dict:
        q, a = C.c_int32(), C.c_int32()
        done = C.c_uint64()
        busy, wall = C.c_double(), C.c_double()
        _check(load().flb_server_stats(self.h, C.byref(q), C.byref(a), C.byref(done),
                                       C.byref(busy), C.byref(wall)), "stats")
        return {"queued": q.value, "active": a.value, "completed": done.value,
                "busy_s": busy.value, "wall_s": wall.value}
