"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: FP64 storage max|df|/max|f| <= 1e-12 after 1000 steps; FP32
shifted storage max|dM~^a|/max|M~^a| <= 1e-5 per moment (f-norm at u0) after
1000 steps; integer-keyed noise must match bit for bit in its uniforms, so
trajectories can only differ by floating-point rounding.
"""
import numpy as np
import pytest

import oracle as O
from paper_1204_6734_amd import inputs as I

pytestmark = pytest.mark.gpu

TAUS = I.mixed_taus(2)
BASES = {"fnorm": (0, 0), "hermite": (1, 1), "lut": (2, 2)}


def both(F, nx, ny, precision, basis=0, **kw):
    g = F.Lattice(F.make_params(nx, ny, precision=precision, basis=basis, **kw))
    o = O.Lattice(O.make_params(nx, ny, basis=basis, **kw))
    return g, o


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("basis", ["fnorm", "hermite", "lut"])
@pytest.mark.parametrize("nx,ny", [(70, 9), (33, 20)])
def test_fp64_trajectory_matches_oracle(flb, basis, nx, ny):
    b = BASES[basis][0]
    kw = dict(rho0=1.0, ux0=0.1, uy0=-0.05, kT=1e-4, tau=TAUS, seed=7, init=2)
    g, o = both(flb, nx, ny, flb.FP64, b, **kw)
    fields = I.random_fields(nx, ny, seed=5, ux0=0.1, uy0=-0.05)
    g.set_fields(*fields)
    o.set_fields(*fields)
    np.testing.assert_allclose(g.populations(), o.populations(), rtol=0, atol=1e-15)
    done = 0
    for n in (1, 1, 3, 95, 900):  # both parities, then long
        g.step(n)
        o.step(n)
        done += n
        err = rel(g.populations(), o.populations())
        assert err <= 1e-12, (basis, done, err)
    assert g.t == o.t == 1000


@pytest.mark.parametrize("basis", ["fnorm", "hermite", "lut"])
def test_fp64_noise_matches_oracle(flb, basis):
    """From equilibrium the first step's change is the noise term alone, so
    comparing f - f^0(rho0, u0) (not f) checks the Gaussians themselves (the
    log, square root, sine and cosine of the Box-Muller transform, eq. (20)
    amplitudes) to 1e-12 relative; the second step checks the odd phase.
    u0 lies away from the midpoints of the table's grid (a velocity exactly
    half-way between two grid points rounds either way)."""
    b = BASES[basis][0]
    nx, ny = 70, 9
    kw = dict(rho0=1.0, ux0=0.08, uy0=-0.025, kT=1e-3, tau=TAUS, seed=21)
    g, o = both(flb, nx, ny, flb.FP64, b, **kw)
    f0 = O.equilibrium(1.0, 0.08, -0.025)[:, None, None]
    for k in range(2):
        g.step(1)
        o.step(1)
        dg, do = g.populations() - f0, o.populations() - f0
        err = rel(dg, do)
        assert err <= 1e-12, (basis, k, err)


def test_table_basis_tie_takes_either_neighbour(flb):
    """The table basis at a local velocity exactly half-way between two grid
    points (Sec. IV, nearest point of the 51 x 51 grid): both neighbours are
    nearest, and which one a rounding of u = j / rho lands on is not fixed by
    the paper.  From an equilibrium at u0 = (0.05, -0.03) (a midpoint on
    both axes) every site's first collision must equal the oracle's
    collision at one of the four neighbouring grid points, to 1e-12; the
    candidates differ by far more than that, so the test tells them apart."""
    nx, ny = 70, 9
    ux0, uy0 = 0.05, -0.03
    kw = dict(rho0=1.0, ux0=ux0, uy0=uy0, kT=1e-3, tau=TAUS, seed=21)
    g = flb.Lattice(flb.make_params(nx, ny, precision=flb.FP64, basis=flb.BASIS_FNORM_LUT,
                                    **kw))
    p = O.make_params(nx, ny, basis=O.BASIS_FNORM_LUT, **kw)
    f0 = O.equilibrium(1.0, ux0, uy0)
    g.step(1)
    fg = g.populations()
    vx, vy, _ = O.velocities()
    # the post-collision value of direction i at x went to x + v_i
    post = np.stack([np.roll(fg[i], (-vy[i], -vx[i]), axis=(0, 1)) for i in range(9)])
    cands = [(ix, iy) for ix in (2, 3) for iy in (-2, -1)]
    spread = 0.0
    for y in range(ny):
        for x in range(nx):
            site = y * nx + x
            outs = [O.collide_lut_at(p, f0, ix, iy, site=site, step=0) for ix, iy in cands]
            spread = max(spread, min(np.abs(outs[0] - o).max() for o in outs[1:]))
            err = min(np.abs(post[:, y, x] - o).max() for o in outs)
            assert err <= 1e-12 * np.abs(f0).max(), (x, y, err)
    assert spread > 1e-6, spread
    # the oracle's own pick is one of the candidates
    mine = O.collide(p, f0, site=0, step=0)
    assert min(np.abs(mine - O.collide_lut_at(p, f0, ix, iy)).max() for ix, iy in cands) == 0.0


# One relaxation time for all six non-conserved modes.  The f-norm collision
# then takes L (M~ / tau) = d / tau without the forward solve and scales the
# Gaussians by the common noise coefficient before their product with L.
ONE_TAU = (0.8,) * 6


@pytest.mark.parametrize("basis", ["fnorm", "lut"])
@pytest.mark.parametrize("sample_every", [0, 1])
def test_one_relaxation_time_fp64_matches_oracle(flb, basis, sample_every):
    """FP64 trajectories from random fields with tau^a = 0.8 for all six
    modes, in the plain and in the sampling step, to 1e-12 at both streaming
    phases and after 1000 steps; then, from equilibrium, the first step's
    change (the noise term alone) to 1e-12."""
    b = BASES[basis][0]
    nx, ny = 70, 9
    kw = dict(rho0=1.0, ux0=0.1, uy0=-0.05, kT=1e-4, tau=ONE_TAU, seed=7, init=2,
              sample_every=sample_every, block_steps=100)
    g, o = both(flb, nx, ny, flb.FP64, b, **kw)
    fields = I.random_fields(nx, ny, seed=5, ux0=0.1, uy0=-0.05)
    g.set_fields(*fields)
    o.set_fields(*fields)
    for n in (1, 1, 3, 95, 900):
        g.step(n)
        o.step(n)
        err = rel(g.populations(), o.populations())
        assert err <= 1e-12, (basis, o.t, err)
    kw = dict(rho0=1.0, ux0=0.08, uy0=-0.025, kT=1e-3, tau=ONE_TAU, seed=21)
    g, o = both(flb, nx, ny, flb.FP64, b, **kw)
    f0 = O.equilibrium(1.0, 0.08, -0.025)[:, None, None]
    for k in range(2):
        g.step(1)
        o.step(1)
        err = rel(g.populations() - f0, o.populations() - f0)
        assert err <= 1e-12, (basis, k, err)


@pytest.mark.parametrize("basis", ["fnorm", "lut"])
@pytest.mark.parametrize("ux0,uy0", [(0.1, 0.0), (0.3, 0.1)])
def test_one_relaxation_time_fp32_matches_oracle(flb, basis, ux0, uy0):
    """FP32-shifted storage with tau^a = 0.8 for all six modes, with the FP32
    collision (u0 = 0.1) and the FP64 one (u0 = 0.3): every moment at u0 to
    1e-5 of its largest value after 1000 steps against the oracle."""
    kw = dict(ux0=ux0, uy0=uy0, kT=FP32_KT[basis], tau=ONE_TAU, seed=11)
    g, o = both(flb, 100, 30, flb.FP32_SHIFTED, BASES[basis][0], **kw)
    g.step(1000)
    o.step(1000)
    mg, mo = g.moments(flb.AT_U0), o.moments(flb.AT_U0)
    worst = max(np.abs(mg[a] - mo[a]).max() / np.abs(mo[a]).max() for a in range(9))
    print(f"{basis} u0 ({ux0}, {uy0}), one tau: worst moment rel err {worst:.2e}")
    assert worst <= 1e-5, worst


@pytest.mark.parametrize("nx,ny", [(3, 3), (3, 17), (65, 3), (64, 4), (4, 65)])
def test_degenerate_shapes_match_oracle(flb, nx, ny):
    """The smallest lattices and thin ones: a single partly filled tile whose
    wavefronts wrap at both ends of a row, a tile row one site high, one
    exact tile, a column of ragged tiles; FP64 f-norm trajectories with noise
    at both streaming phases to 1e-12, and zero steps leave the state and
    the clock alone."""
    kw = dict(rho0=1.0, ux0=0.1, uy0=-0.05, kT=1e-4, tau=TAUS, seed=31, init=2)
    g, o = both(flb, nx, ny, flb.FP64, 0, **kw)
    fields = I.random_fields(nx, ny, seed=9, ux0=0.1, uy0=-0.05)
    g.set_fields(*fields)
    o.set_fields(*fields)
    f0 = g.populations()
    g.step(0)
    assert g.t == 0
    np.testing.assert_array_equal(g.populations(), f0)
    for n in (1, 1, 7):
        g.step(n)
        o.step(n)
        err = rel(g.populations(), o.populations())
        assert err <= 1e-12, (nx, ny, o.t, err)


def test_fp64_moments_match_oracle(flb):
    kw = dict(ux0=0.15, kT=1e-4, tau=TAUS, seed=3)
    g, o = both(flb, 45, 21, flb.FP64, **kw)
    g.step(37)
    o.step(37)
    for at in (flb.AT_LOCAL, flb.AT_U0, flb.AT_HERMITE):
        mg, mo = g.moments(at), o.moments(at)
        for a in range(9):
            scale = max(np.abs(mo[a]).max(), 1e-3)
            assert np.abs(mg[a] - mo[a]).max() <= 1e-12 * scale, (at, a)


# Noise temperature of the FP32 parity runs per basis.  The table basis is a
# step function of the local velocity (nearest point of a grid of spacing
# 0.02): an FP32 trajectory carries the local velocity to ~1e-8 of the FP64
# one, so a site within that distance of a grid midpoint may round to the
# other grid point, whose basis projects the noise differently.  At
# kT = 1e-4 the velocity spreads by sqrt(kT / rho0) = 0.01, half the grid
# spacing, and a 1000-step run meets tens of such sites; at kT = 1e-6 the
# spread is 1e-3 and the midpoints (0.01 away from the grid velocities u0
# used here) lie ten standard deviations out.
FP32_KT = {"fnorm": 1e-4, "hermite": 1e-4, "lut": 1e-6}


@pytest.mark.parametrize("basis", ["fnorm", "hermite", "lut"])
@pytest.mark.parametrize("ux0", [0.0, 0.1, 0.2])
def test_fp32_shifted_moments_match_fp64_oracle(flb, basis, ux0):
    """FP32-shifted storage with the FP32 collision (|u0| <= 0.25) in each
    basis (local f-norm of Sec. IV, Hermite norm of App. A, table basis of
    Sec. IV), against the FP64 oracle: every moment at u0 to 1e-5 of its
    largest value after 1000 steps."""
    nx, ny = 100, 30
    kw = dict(ux0=ux0, kT=FP32_KT[basis], tau=TAUS, seed=11)
    g, o = both(flb, nx, ny, flb.FP32_SHIFTED, BASES[basis][0], **kw)
    g.step(1000)
    o.step(1000)
    mg, mo = g.moments(flb.AT_U0), o.moments(flb.AT_U0)
    worst = max(np.abs(mg[a] - mo[a]).max() / np.abs(mo[a]).max() for a in range(9))
    print(f"{basis} u0 {ux0}: worst moment rel err {worst:.2e}")
    assert worst <= 1e-5, worst


@pytest.mark.parametrize("basis", ["fnorm", "hermite", "lut"])
def test_fp32_storage_fp64_compute_matches_oracle(flb, basis):
    """|u0| above 0.25: FP32-shifted storage with the collision computed in
    FP64 (the large-velocity path), against the oracle after 1000 steps."""
    b = {"fnorm": flb.BASIS_FNORM_LOCAL, "hermite": flb.BASIS_HERMITE,
         "lut": flb.BASIS_FNORM_LUT}[basis]
    nx, ny = 100, 30
    kw = dict(ux0=0.3, uy0=0.1, kT=1e-4, tau=TAUS, seed=12)
    g, o = both(flb, nx, ny, flb.FP32_SHIFTED, basis=b, **kw)
    g.step(1000)
    o.step(1000)
    mg, mo = g.moments(flb.AT_U0), o.moments(flb.AT_U0)
    worst = max(np.abs(mg[a] - mo[a]).max() / np.abs(mo[a]).max() for a in range(9))
    assert worst <= 1e-5, worst


@pytest.mark.parametrize("basis,ux0", [("fnorm", 0.1), ("fnorm", 0.3), ("hermite", 0.1),
                                       ("hermite", 0.2), ("lut", 0.1), ("lut", 0.2)])
def test_fp32_covariance_sums_match_oracle(flb, basis, ux0):
    """FP32-shifted storage (FP32 and, at u0 = 0.3, FP64 collisions) in each
    basis: the correlator sums, staged in FP32 and summed on the matrix
    cores, against the oracle's FP64 run of the same noise.  The stored
    deviations h carry one FP32 rounding (2^-24 relative) and the
    dissipative update does not amplify it, so the covariances, products of
    two deviations, agree to a few 1e-7 of their largest entry (bound 1e-6),
    and the means to 1e-6 of the fluctuation amplitude sqrt(max_i C_ii), the
    scale of a first moment.  (Measured against the means' own size instead,
    the error grows as kT falls, since the means nearly cancel: 1.2e-6 at
    kT = 1e-4, 1.3e-5 at 1e-6.)"""
    kw = dict(ux0=ux0, kT=FP32_KT[basis], tau=TAUS, seed=5, sample_every=1, block_steps=50)
    g, o = both(flb, 40, 24, flb.FP32_SHIFTED, BASES[basis][0], **kw)
    g.step(300)
    o.step(300)
    cg, co = g.covariance(), o.covariance()
    assert cg["nsamples"] == co["nsamples"] == 300 * 40 * 24
    scale = np.abs(co["cov_f"]).max()
    err = np.abs(cg["cov_f"] - co["cov_f"]).max() / scale
    sigma = np.sqrt(np.diag(co["cov_f"]).max())
    merr = np.abs(cg["mean_df"] - co["mean_df"]).max() / sigma
    print(f"{basis} u0 {ux0}: cov_f rel err {err:.2e}, mean_df err / sigma {merr:.2e}")
    assert err <= 1e-6 and merr <= 1e-6, (err, merr)


def test_time_blocks_of_many_tiles_match_oracle(flb):
    """Closing a time block folds ranges of tiles in parallel: 520 x 140 is
    9 x 35 = 315 tiles, so ranges hold two tiles and the last one is short.
    Five blocks close in 50 samples; sums and standard errors against the
    oracle's serial ones."""
    kw = dict(ux0=0.1, kT=1e-4, tau=TAUS, seed=17, sample_every=1, block_steps=10)
    g, o = both(flb, 520, 140, flb.FP64, **kw)
    g.step(50)
    o.step(50)
    cg, co = g.covariance(), o.covariance()
    assert cg["nsamples"] == co["nsamples"] == 50 * 520 * 140
    assert cg["nblocks"] == co["nblocks"] == 5
    for key in ("cov_f", "cov_m_fnorm_u0", "se_cov_f"):
        err = np.abs(cg[key] - co[key]).max() / np.abs(co[key]).max()
        assert err <= 1e-10, (key, err)


def test_covariance_sums_match_oracle(flb):
    kw = dict(ux0=0.1, kT=1e-4, tau=TAUS, seed=5, sample_every=1, block_steps=50)
    g, o = both(flb, 40, 24, flb.FP64, **kw)
    g.step(300)
    o.step(300)
    cg, co = g.covariance(), o.covariance()
    assert cg["nsamples"] == co["nsamples"] == 300 * 40 * 24
    assert cg["nblocks"] == co["nblocks"] == 6
    for k in ("mean_df", "cov_f", "cov_m_fnorm_u0", "cov_m_hermite", "se_cov_f"):
        assert np.abs(cg[k] - co[k]).max() <= 1e-10 * np.abs(co[k]).max(), k


def test_time_block_merge_matches_oracle(flb):
    """More closed blocks than the record list holds: pairs merge, length doubles."""
    kw = dict(kT=1e-4, seed=5, sample_every=1, block_steps=1)
    g, o = both(flb, 8, 8, flb.FP64, **kw)
    g.step(1030)
    o.step(1030)
    cg, co = g.covariance(), o.covariance()
    assert cg["nblocks"] == co["nblocks"]
    for k in ("cov_f", "se_cov_f", "se_cov_m"):
        assert np.abs(cg[k] - co[k]).max() <= 1e-9 * np.abs(co[k]).max(), k


@pytest.mark.parametrize("prec,nx,ny", [("fp64", 16, 8), ("fp64", 12, 10), ("fp64", 64, 32),
                                         ("fp64", 8, 1024), ("fp32", 64, 32), ("fp32", 12, 10),
                                         ("fp32", 256, 16), ("fp32", 96, 40), ("fp64", 40, 96),
                                         ("fp32", 128, 64)])
def test_structure_factor_matches_oracle(flb, prec, nx, ny):
    """S(k) of all five kinds against the oracle: FFT sizes from 8 to 1024
    (radix-8 passes after a radix-2 or -4 one), direct DFTs for other
    sizes; transposes of several 32 x 32 tiles both ways, unequal in number
    and ragged at the far edges (96 x 40, 40 x 96, 128 x 64), which the
    diagonal tile order visits once each.  FP32-shifted lattices transform
    in FP32 (accumulators FP64)."""
    precision = flb.FP64 if prec == "fp64" else flb.FP32_SHIFTED
    tol = 1e-10 if prec == "fp64" else 2e-5
    kw = dict(ux0=0.1, kT=1e-4, seed=9, sk_every=3)
    g, o = both(flb, nx, ny, precision, **kw)
    g.step(40)
    o.step(40)
    scale = np.abs(o.structure_factor(0)).max()
    for w in range(5):
        sg, so = g.structure_factor(w), o.structure_factor(w)
        assert np.abs(sg - so).max() <= tol * scale, w


def test_fourier_mode_matches_oracle(flb):
    nx, ny = 48, 10
    g, o = both(flb, nx, ny, flb.FP64, ux0=0.1, kT=0.0, init=2)
    fields = I.shear_wave_fields(nx, ny, ux0=0.1, amp=1e-3)
    g.set_fields(*fields)
    o.set_fields(*fields)
    g.step(11)
    o.step(11)
    for which, kx, ky in [(2, 1, 0), (0, 3, 2), (1, 47, 9)]:
        a, b = g.fourier_mode(which, kx, ky), o.fourier_mode(which, kx, ky)
        assert abs(a - b) <= 1e-12 * max(1e-3, abs(b)) * nx * ny


@pytest.mark.parametrize("prec,nx,ny", [("fp64", 48, 10), ("fp64", 300, 7), ("fp32", 300, 7),
                                         ("fp32", 8192, 8), ("fp64", 262500, 3)])
def test_fourier_mode_of_the_gpu_state(flb, prec, nx, ny):
    """The readback of one Fourier coefficient of d rho, dj~_x, dj~_y against
    the oracle's coefficient (the separable sum by its definition) of the
    GPU's own populations, at both streaming phases: one partly filled block
    of 256 columns, two with a ragged second, the benchmark's row length, and
    more column blocks than the readback has partials (a thread then walks
    several columns); ky = 0 and ky != 0."""
    ux0, uy0 = 0.1, -0.05
    precision = flb.FP64 if prec == "fp64" else flb.FP32_SHIFTED
    g = flb.Lattice(flb.make_params(nx, ny, precision=precision, ux0=ux0, uy0=uy0, kT=1e-4,
                                    seed=5, init=2))
    g.set_fields(*I.random_fields(nx, ny, seed=3, ux0=ux0, uy0=uy0))
    modes = [(2, 1, 0), (0, 3, 2), (1, nx - 1, ny - 1), (2, 0, 0), (1, nx // 2, 1)]
    for _ in range(2):  # odd phase, then even phase
        g.step(1)
        fields = O.sk_fields(g.populations(), 1.0, ux0, uy0)
        for which, kx, ky in modes:
            a = g.fourier_mode(which, kx, ky)
            b = O.fourier_coefficient(fields[which], kx, ky)
            scale = np.abs(fields[which]).sum()
            assert abs(a - b) <= 1e-12 * scale, (prec, nx, ny, g.t, which, kx, ky, a, b)


def test_thermal_start_matches_oracle(flb):
    kw = dict(ux0=0.05, kT=1e-3, seed=21, init=1)
    g, o = both(flb, 20, 12, flb.FP64, **kw)
    assert rel(g.populations(), o.populations()) <= 1e-14


def test_checkpoint_restore_is_bit_identical(flb):
    for prec in (flb.FP64, flb.FP32_SHIFTED):
        p = flb.make_params(50, 17, precision=prec, ux0=0.1, kT=1e-4, tau=TAUS, seed=4)
        a = flb.Lattice(p)
        a.step(37)
        b = flb.Lattice(p)
        b.step(20)
        blob = b.checkpoint()
        c = flb.Lattice(p)
        c.restore(blob)
        assert c.t == 20
        c.step(17)
        np.testing.assert_array_equal(a.populations(), c.populations())
        # another reference state cannot take these offsets; another kT can
        other = flb.make_params(50, 17, precision=prec, ux0=0.11, kT=1e-4, tau=TAUS, seed=4)
        with pytest.raises(flb.FlbError) as e:
            flb.Lattice(other).restore(blob)
        assert e.value.code == flb.E_ARG
        hot = flb.Lattice(flb.make_params(50, 17, precision=prec, ux0=0.1, kT=2e-4, tau=TAUS,
                                          seed=4))
        hot.restore(blob)
        np.testing.assert_array_equal(hot.populations(), b.populations())


def test_in_place_streaming_preserves_mass_and_momentum(flb):
    p = flb.make_params(37, 23, precision=flb.FP64, ux0=0.1, kT=1e-3, tau=TAUS, seed=2)
    L = flb.Lattice(p)
    f0 = L.populations()
    L.step(501)
    f1 = L.populations()
    vx, vy, _ = O.velocities()
    for w in (np.ones(9), vx, vy):
        a = np.tensordot(w, f0, axes=(0, 0)).sum()
        b = np.tensordot(w, f1, axes=(0, 0)).sum()
        assert abs(a - b) <= 1e-10 * f0.sum()


def test_invalid_velocity_is_reported(flb):
    nx, ny = 20, 8
    L = flb.Lattice(flb.make_params(nx, ny, precision=flb.FP64, init=2))
    rho, ux, uy = np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx))
    ux[3, 5] = 0.9
    L.set_fields(rho, ux, uy)
    L.step(2)
    with pytest.raises(flb.FlbError) as e:
        L.sync()
    assert e.value.code == flb.E_INVALID_VELOCITY and L.error_step == 0
    with pytest.raises(flb.FlbError) as e:
        flb.Lattice(flb.make_params(16, 16, ux0=0.5, uy0=0.5))
    assert e.value.code == flb.E_INVALID_VELOCITY


def test_create_on_caller_buffer(flb):
    import torch
    p = flb.make_params(64, 40, precision=flb.FP32_SHIFTED, ux0=0.1, kT=1e-4, seed=8)
    nbytes = flb.Lattice.bytes_needed(p)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream()
    a = flb.Lattice(p, stream=s, device_buffer=(buf.data_ptr(), nbytes))
    b = flb.Lattice(p)
    a.step(25)
    b.step(25)
    np.testing.assert_array_equal(a.populations(), b.populations())
