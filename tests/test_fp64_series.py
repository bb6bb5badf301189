"""The polynomial coefficients of the FP64 Box-Muller transform
(`paper_1204_6734_amd/csrc/fp64_series.hpp`), checked on the CPU against
long-double sin, cos and artanh at the arguments the transform meets: every
reduced angle r = pi k 2^-21, k = 0 .. 2^19, of the 21-bit draw, and a dense
grid of z over |z| <= (sqrt2 - 1)/(sqrt2 + 1) for ln m = 2 artanh z.  The
polynomials are evaluated as the device does (Horner with fused
multiply-adds, emulated in long double and rounded to FP64 at each step) and
must agree to within 1.5 ulp of the FP64 result; the committed header must be
what its generator writes."""
import importlib.util
import os
import re

import numpy as np

ROOT = os.path.join(os.path.dirname(__file__), "..")
CSRC = os.path.join(ROOT, "paper_1204_6734_amd", "csrc")
LD = np.longdouble


def coefficients():
    text = open(os.path.join(CSRC, "fp64_series.hpp")).read()
    out = {}
    for name, body in re.findall(r"constexpr double (\w+)\[\d+\] = \{([^}]*)\};", text):
        out[name] = [float(v) for v in body.split(",")]
    return out


def horner_fma(c, x):
    """Horner with one rounding to FP64 per fused multiply-add."""
    p = np.full(x.shape, c[-1], dtype=np.float64)
    for ck in reversed(c[:-1]):
        p = (p.astype(LD) * x.astype(LD) + LD(ck)).astype(np.float64)
    return p


def ulp_error(got, want):
    return np.abs(got.astype(LD) - want) / np.spacing(np.abs(want).astype(np.float64)).astype(LD)


def test_header_is_generated():
    spec = importlib.util.spec_from_file_location("gen_fp64_series",
                                                  os.path.join(CSRC, "gen_fp64_series.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    assert gen.header_text() == open(os.path.join(CSRC, "fp64_series.hpp")).read()


def test_sin_cos_at_every_reduced_angle():
    c = coefficients()
    assert c["kSinSeries"][0] == 1.0 and c["kCosSeries"][0] == 1.0
    k = np.arange(0, (1 << 19) + 1, dtype=np.float64)
    r = k * (np.pi / float(1 << 21))  # as the device forms it: one rounding
    r2 = r * r
    s = r * horner_fma(c["kSinSeries"], r2)
    co = horner_fma(c["kCosSeries"], r2)
    rl = r.astype(LD)
    es, ec = ulp_error(s[1:], np.sin(rl)[1:]), ulp_error(co, np.cos(rl))
    assert es.max() <= 1.5 and ec.max() <= 1.5, (float(es.max()), float(ec.max()))


def test_artanh_over_the_reduced_interval():
    c = coefficients()
    assert c["kAtanhSeries"][0] == 1.0
    zmax = (np.sqrt(2.0) - 1) / (np.sqrt(2.0) + 1)
    z = np.linspace(-zmax, zmax, 1_000_001)
    z = z[z != 0]
    a = z * horner_fma(c["kAtanhSeries"], z * z)
    err = ulp_error(a, np.arctanh(z.astype(LD)))
    assert err.max() <= 1.5, float(err.max())
