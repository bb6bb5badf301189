"""Host-side checks of the C-ABI library: it loads without a GPU, exports
every entry point include/flb.h declares, and its ctypes structures match
the header's layout.  No compute calls (no GPU here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "flb.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|size_t|uint64_t|int64_t|void|char)\s*\**\s*"
                       r"(flb3?_\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("flb_lattice_create", "flb_lattice_step", "flb_lattice_read_moments",
                 "flb_lattice_read_covariance", "flb_ensemble_step", "flb_server_submit"):
        assert must in names
    assert len(names) >= 40


def test_library_exports_every_declared_symbol():
    import paper_1204_6734_amd as F
    lib = F.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layouts():
    import paper_1204_6734_amd as F
    # flb_params: 2 int32, 4 doubles, 6 doubles, uint64, 6 int32
    assert C.sizeof(F.Params) == 8 + 8 * 4 + 8 * 6 + 8 + 4 * 6
    assert F.Params.tau.offset == 40 and F.Params.seed.offset == 88
    assert C.sizeof(F.Cov) == 16 + 8 * (9 + 81 * 6)
    assert F.Result.cov.offset == 56


def test_create_without_gpu_fails_cleanly():
    import paper_1204_6734_amd as F
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("GPU present")
    except Exception:
        pass
    with pytest.raises(F.FlbError) as e:
        F.Lattice(F.make_params(16, 16))
    assert e.value.code in (F.E_OOM, F.E_HIP)


def test_argument_errors_are_reported():
    import paper_1204_6734_amd as F
    lib = F.load()
    bad = [F.make_params(2, 16), F.make_params(16, 16, tau=(0.5,) * 6),
           F.make_params(16, 16, kT=-1.0), F.make_params(16, 16, ux0=0.5, uy0=0.5)]
    codes = []
    for p in bad:
        h = C.c_void_p()
        codes.append(lib.flb_lattice_create(C.byref(p), None, C.byref(h)))
        assert lib.flb_last_error()
    assert codes[:3] == [F.E_ARG] * 3 and codes[3] == F.E_INVALID_VELOCITY
    assert lib.flb_lattice_bytes(C.byref(bad[0])) == 0
    assert lib.flb_lattice_bytes(C.byref(F.make_params(64, 64))) > 9 * 64 * 64 * 4


def test_launch_config_layout_and_null_handles():
    import paper_1204_6734_amd as F
    lib = F.load()
    assert C.sizeof(F.LaunchConfig) == 16 and F.LaunchConfig.ms_per_step.offset == 8
    c = F.LaunchConfig(2, 64, 0.0)
    n = C.c_int32()
    assert lib.flb_lattice_autotune(None, 3, None, 0, C.byref(n)) == F.E_ARG
    assert lib.flb_ensemble_autotune(None, 3, None, 0, C.byref(n)) == F.E_ARG
    assert lib.flb_lattice_set_launch(None, C.byref(c)) == F.E_ARG
    assert lib.flb_ensemble_get_launch(None, C.byref(c)) == F.E_ARG


def test_d3q19_struct_layouts_and_argument_errors():
    import paper_1204_6734_amd as F
    lib = F.load()
    assert C.sizeof(F.Params3) == 8 * 4 + 8 * 5 + 8 * 15 + 8
    assert F.Params3.rho0.offset == 32 and F.Params3.seed.offset == 192
    assert C.sizeof(F.Cov3) == 16 + 8 * (19 + 361 * 2)
    h = C.c_void_p()
    bad = [F.make_params3(2, 4, 4), F.make_params3(4, 4, 4, tau=(0.5,)),
           F.make_params3(4, 4, 4, basis=F.BASIS_FNORM_LUT), F.make_params3(4, 4, 4, kT=-1.0),
           F.make_params3(4, 4, 4, ux0=0.6, uy0=0.6)]
    codes = [lib.flb3_lattice_create(C.byref(p), None, C.byref(h)) for p in bad]
    assert codes[:4] == [F.E_ARG] * 4 and codes[4] == F.E_INVALID_VELOCITY
    assert lib.flb3_lattice_step(None, 1) == F.E_ARG


def test_largest_lattice_bound():
    """Sizes are checked on the host: 9 ny P < 2^32 elements with P = nx
    rounded up to 64 (the row pitch of the population storage)."""
    import paper_1204_6734_amd as F
    lib = F.load()
    for prec in (F.FP64, F.FP32_SHIFTED):
        ok = F.make_params(21824, 21824, precision=prec)
        bad = F.make_params(21825, 21824, precision=prec)
        assert lib.flb_lattice_bytes(C.byref(ok)) >= 9 * 21824 * 21824 * (8 if prec == F.FP64
                                                                             else 4)
        assert lib.flb_lattice_bytes(C.byref(bad)) == 0


def test_server_request_bytes_follow_the_server_precision():
    """A request is stored in the server's precision whatever its own
    precision field says; the sizing call charges what admission charges."""
    import paper_1204_6734_amd as F
    p = F.make_params(512, 512, precision=F.FP64, sample_every=1)
    b32 = F.Server.request_bytes(p, precision=F.FP32_SHIFTED)
    b64 = F.Server.request_bytes(p, precision=F.FP64)
    pops = 9 * 512 * 512
    assert b32 >= 4 * pops and b64 >= 8 * pops and b64 - b32 == 4 * pops
    assert F.Server.request_bytes(F.make_params(2, 512)) == 0


def test_copy_probe_argument_errors():
    """Rejected before any device call (no GPU needed)."""
    import paper_1204_6734_amd as F
    lib = F.load()
    ms = C.c_double()
    for args in [(2, 64, 1, 5), (64, 2, 1, 5), (64, 64, 7, 5), (64, 64, 1, 0), (64, 64, 1, 1001),
                 (1 << 20, 1 << 20, 1, 5)]:
        assert lib.flb_copy_probe(*args, C.byref(ms)) == F.E_ARG, args
    assert lib.flb_copy_probe(64, 64, 1, 5, None) == F.E_ARG
    for args in [(0, 5), (24, 5), (1 << 40, 5), (1024, 0)]:
        assert lib.flb_stream_copy_probe(*args, C.byref(ms)) == F.E_ARG, args
    assert lib.flb_stream_copy_probe(1024, 5, None) == F.E_ARG


def test_host_arrays_are_size_checked_before_the_call():
    """The library reads exactly 9 nx ny (or nx ny) doubles from the pointer it
    is given; the binding refuses arrays of another size."""
    import numpy as np
    import paper_1204_6734_amd as F
    ok = F._host_f64(np.zeros((9, 4, 5), np.float32), 180, "t")
    assert ok.dtype == np.float64 and ok.flags.c_contiguous and ok.size == 180
    with pytest.raises(ValueError):
        F._host_f64(np.zeros((9, 4, 4)), 180, "t")
    with pytest.raises(ValueError):
        F._host_f64(np.zeros(181), 180, "t")
