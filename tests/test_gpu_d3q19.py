"""D3Q19 lattices on the GPU against the D3Q19 oracle (the generalisation
of Sec. V; model in include/flb.h): FP64 trajectories to 1e-12 at both
streaming phases for the local f-norm and the Hermite rows, FP32-shifted
storage to 1e-5 on the fluctuations, correlator sums, conservation, and the
ideal-gas covariance at rest within standard errors."""
import math

import numpy as np
import pytest

from oracle import d3q19 as D

pytestmark = pytest.mark.gpu

TAUS = tuple(np.round(np.random.default_rng(2).uniform(0.6, 1.5, 15), 6))


def both(F, nx, ny, nz, precision, basis, **kw):
    g = F.Lattice3(F.make_params3(nx, ny, nz, precision=precision, basis=basis, **kw))
    o = D.Lattice(D.make_params(nx, ny, nz, basis=basis, **kw))
    return g, o


def perturbed(nx, ny, nz, u0, seed=1):
    """Local equilibria with 1 % density and velocity perturbations."""
    rng = np.random.default_rng(seed)
    rho = 1 + 0.01 * rng.standard_normal((nz, ny, nx))
    u = [u0[a] + 0.01 * rng.standard_normal((nz, ny, nx)) for a in range(3)]
    vx, vy, vz, w = D.velocities()
    f = np.empty((19, nz, ny, nx))
    uu = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    for i in range(19):
        cu = vx[i] * u[0] + vy[i] * u[1] + vz[i] * u[2]
        f[i] = w[i] * rho * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * uu)
    return f


@pytest.mark.parametrize("basis", ["fnorm", "hermite"])
def test_fp64_trajectory_matches_oracle(flb, basis):
    b = flb.BASIS_FNORM_LOCAL if basis == "fnorm" else flb.BASIS_HERMITE
    nx, ny, nz = 70, 6, 5  # two tiles along x, the second ragged
    kw = dict(ux0=0.1, uy0=-0.05, uz0=0.03, kT=1e-4, tau=TAUS, seed=9)
    g, o = both(flb, nx, ny, nz, flb.FP64, b, **kw)
    f = perturbed(nx, ny, nz, (0.1, -0.05, 0.03))
    g.set_populations(f)
    o.set_populations(f)
    for n in (1, 1, 23):
        g.step(n)
        o.step(n)
        fg, fo = g.populations(), o.populations()
        err = np.abs(fg - fo).max() / np.abs(fo).max()
        assert err <= 1e-12, (basis, o.t, err)


@pytest.mark.parametrize("basis", ["fnorm", "hermite"])
def test_fp64_noise_matches_oracle(flb, basis):
    """From equilibrium the first step's change is the noise term alone:
    f - f^0(rho0, u0) checks the fifteen Gaussians per site to 1e-12
    relative, at both streaming phases."""
    b = flb.BASIS_FNORM_LOCAL if basis == "fnorm" else flb.BASIS_HERMITE
    nx, ny, nz = 70, 5, 4
    kw = dict(ux0=0.08, uy0=-0.03, uz0=0.02, kT=1e-3, tau=TAUS, seed=23)
    g, o = both(flb, nx, ny, nz, flb.FP64, b, **kw)
    f0 = D.equilibrium(1.0, 0.08, -0.03, 0.02)[:, None, None, None]
    for k in range(2):
        g.step(1)
        o.step(1)
        dg, do = g.populations() - f0, o.populations() - f0
        err = np.abs(dg - do).max() / np.abs(do).max()
        assert err <= 1e-12, (basis, k, err)


@pytest.mark.parametrize("shape", [(3, 3, 3), (3, 5, 4), (65, 3, 3)])
def test_degenerate_shapes_match_oracle(flb, shape):
    """The smallest lattice and thin ones (rows that wrap inside one
    wavefront, a ragged second tile), FP64 f-norm with noise, both phases."""
    nx, ny, nz = shape
    kw = dict(ux0=0.1, uy0=-0.05, uz0=0.03, kT=1e-4, tau=TAUS, seed=13)
    g, o = both(flb, nx, ny, nz, flb.FP64, flb.BASIS_FNORM_LOCAL, **kw)
    f = perturbed(nx, ny, nz, (0.1, -0.05, 0.03), seed=4)
    g.set_populations(f)
    o.set_populations(f)
    for n in (1, 1, 5):
        g.step(n)
        o.step(n)
        fg, fo = g.populations(), o.populations()
        assert np.abs(fg - fo).max() <= 1e-12 * np.abs(fo).max(), (shape, o.t)


@pytest.mark.parametrize("basis", ["fnorm", "hermite"])
def test_fp32_shifted_matches_fp64_oracle(flb, basis):
    """FP32-shifted storage with the FP32 collision of either basis (the
    Hermite-type rows draw their Gaussians inside the collision, with the
    local density in the Box-Muller radius): the fluctuations f - f^0(rho0,
    u0) after 200 steps to 1e-5 of their largest value, at 70 x 8 x 6 (a
    ragged second tile along x)."""
    b = flb.BASIS_FNORM_LOCAL if basis == "fnorm" else flb.BASIS_HERMITE
    nx, ny, nz = 70, 8, 6
    kw = dict(ux0=0.1, uy0=0.05, uz0=-0.02, kT=1e-4, tau=TAUS, seed=3)
    g, o = both(flb, nx, ny, nz, flb.FP32_SHIFTED, b, **kw)
    g.step(200)
    o.step(200)
    f0 = D.equilibrium(1.0, 0.1, 0.05, -0.02)[:, None, None, None]
    dg, do = g.populations() - f0, o.populations() - f0
    err = np.abs(dg - do).max() / np.abs(do).max()
    print(f"{basis}: max |df_gpu - df_oracle| / max |df| = {err:.2e}")
    assert err <= 1e-5, (basis, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_relaxation_time_matches_oracle(flb, prec):
    """All fifteen relaxation times equal (0.8): the f-norm collision takes
    L (M~ / tau) = d / tau without the forward solve and scales the
    Gaussians by the common coefficient.  FP64 against the oracle to 1e-12
    from perturbed equilibria at both streaming phases; FP32-shifted storage
    on the fluctuations to 1e-5 after 200 steps."""
    nx, ny, nz = 70, 6, 5
    kw = dict(ux0=0.1, uy0=-0.05, uz0=0.03, kT=1e-4, tau=(0.8,) * 15, seed=9)
    if prec == "fp64":
        g, o = both(flb, nx, ny, nz, flb.FP64, flb.BASIS_FNORM_LOCAL, **kw)
        f = perturbed(nx, ny, nz, (0.1, -0.05, 0.03))
        g.set_populations(f)
        o.set_populations(f)
        for n in (1, 1, 23):
            g.step(n)
            o.step(n)
            fg, fo = g.populations(), o.populations()
            err = np.abs(fg - fo).max() / np.abs(fo).max()
            assert err <= 1e-12, (o.t, err)
    else:
        g, o = both(flb, nx, ny, nz, flb.FP32_SHIFTED, flb.BASIS_FNORM_LOCAL, **kw)
        g.step(200)
        o.step(200)
        f0 = D.equilibrium(1.0, 0.1, -0.05, 0.03)[:, None, None, None]
        dg, do = g.populations() - f0, o.populations() - f0
        err = np.abs(dg - do).max() / np.abs(do).max()
        print(f"one tau: max |df_gpu - df_oracle| / max |df| = {err:.2e}")
        assert err <= 1e-5, err


@pytest.mark.parametrize("basis", ["fnorm", "hermite"])
def test_fp32_correlator_sums_match_oracle(flb, basis):
    """The correlator sums of an FP32-shifted lattice (values staged in FP32,
    products and sums in FP64 on the matrix cores) against the oracle's FP64
    run of the same noise: the stored deviations carry one FP32 rounding, so
    the covariances agree to a few 1e-7 of their largest entry (bound 1e-6)
    and the means to 1e-6 of the fluctuation amplitude sqrt(max_i C_ii)."""
    b = flb.BASIS_FNORM_LOCAL if basis == "fnorm" else flb.BASIS_HERMITE
    nx, ny, nz = 20, 5, 4
    kw = dict(ux0=0.08, uy0=-0.02, kT=1e-4, tau=TAUS, seed=21, sample_every=1, block_steps=5)
    g, o = both(flb, nx, ny, nz, flb.FP32_SHIFTED, b, **kw)
    g.step(30)
    o.step(30)
    cg, co = g.covariance(), o.covariance()
    assert cg["nsamples"] == co["nsamples"] == 30 * nx * ny * nz
    assert cg["nblocks"] == co["nblocks"] == 6
    err = np.abs(cg["cov_f"] - co["cov_f"]).max() / np.abs(co["cov_f"]).max()
    sigma = math.sqrt(np.diag(co["cov_f"]).max())
    merr = np.abs(cg["mean_df"] - co["mean_df"]).max() / sigma
    print(f"{basis}: cov_f rel err {err:.2e}, mean_df err / sigma {merr:.2e}")
    assert err <= 1e-6 and merr <= 1e-6, (basis, err, merr)


def test_correlator_sums_match_oracle(flb):
    nx, ny, nz = 20, 5, 4
    kw = dict(ux0=0.08, kT=1e-4, tau=TAUS, seed=21, sample_every=1, block_steps=5)
    g, o = both(flb, nx, ny, nz, flb.FP64, flb.BASIS_FNORM_LOCAL, **kw)
    g.step(30)
    o.step(30)
    cg, co = g.covariance(), o.covariance()
    assert cg["nsamples"] == co["nsamples"] == 30 * nx * ny * nz
    assert cg["nblocks"] == co["nblocks"] == 6
    for k in ("mean_df", "cov_f", "se_cov_f"):
        assert np.abs(cg[k] - co[k]).max() <= 1e-10 * np.abs(co[k]).max(), k


def test_conservation_fp64(flb):
    nx, ny, nz = 33, 7, 5
    L = flb.Lattice3(flb.make_params3(nx, ny, nz, precision=flb.FP64, ux0=0.12, uz0=-0.04,
                                      kT=1e-3, tau=TAUS, seed=4))
    vx, vy, vz, _ = D.velocities()
    f = L.populations()
    m0 = f.sum()
    j0 = [np.tensordot(v, f, axes=(0, 0)).sum() for v in (vx, vy, vz)]
    L.step(100)
    f = L.populations()
    assert abs(f.sum() - m0) < 1e-11 * m0
    for v, j in zip((vx, vy, vz), j0):
        assert abs(np.tensordot(v, f, axes=(0, 0)).sum() - j) < 1e-11 * m0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_statistics_at_rest_match_closed_form(flb, prec):
    """5^3 lattice (odd sides: only the k = 0 mass and momentum are
    invariant), u0 = 0: <df_i df_j> = mu rho0 [w_i delta_ij - w_i w_j
    (1 + 3 v_i.v_j) / N] within standard errors."""
    precision = flb.FP64 if prec == "fp64" else flb.FP32_SHIFTED
    n, kT = 5, 1e-4
    L = flb.Lattice3(flb.make_params3(n, n, n, precision=precision, kT=kT, seed=8,
                                      sample_every=1, block_steps=500))
    L.step(500)
    L.reset_stats()
    L.step(20000)
    c = L.covariance()
    vx, vy, vz, w = D.velocities()
    C = np.stack([vx, vy, vz], axis=1).astype(float)
    want = 3 * kT * (np.diag(w) - np.outer(w, w) * (1 + 3 * C @ C.T) / n ** 3)
    iu = np.triu_indices(19)
    z = ((c["cov_f"] - want) / c["se_cov_f"])[iu]
    zmax, zrms = np.abs(z).max(), math.sqrt((z ** 2).mean())
    print(f"D3Q19 5^3 {prec} at rest: max|z| {zmax:.2f} rms {zrms:.2f}")
    assert zmax < 4.5 and 0.5 < zrms < 1.6, (zmax, zrms)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_invalid_velocity_is_reported(flb, prec):
    """A site outside the region where the f-norm exists (some g_i <= 0,
    Fig. 11; here the rest weight at u = (0.9, 0, 0)) sets the lattice's
    error flag with the first failing step; the launch itself completes."""
    precision = flb.FP64 if prec == "fp64" else flb.FP32_SHIFTED
    nx, ny, nz = 70, 5, 4
    L = flb.Lattice3(flb.make_params3(nx, ny, nz, precision=precision, kT=1e-4, seed=2))
    f = perturbed(nx, ny, nz, (0.0, 0.0, 0.0))
    vx, vy, vz, w = D.velocities()
    f[:, 2, 3, 66] = [w[i] * (1 + 3 * 0.9 * vx[i] + 4.5 * (0.9 * vx[i]) ** 2 - 1.5 * 0.81)
                      for i in range(19)]
    L.set_populations(f, 5)
    L.step(3)
    with pytest.raises(flb.FlbError) as e:
        L.sync()
    assert e.value.code == flb.E_INVALID_VELOCITY and L.error_step == 5


def one_step_samples3(po, f0, t, sites, nx, ny, nz):
    """Oracle value of f_i(x, t+1) = collide(f(x - v_i, t))_i for sampled x."""
    vx, vy, vz, _ = D.velocities()
    out = np.empty((len(sites), 19))
    for k, (x, y, z) in enumerate(sites):
        for i in range(19):
            xs, ys, zs = (x - vx[i]) % nx, (y - vy[i]) % ny, (z - vz[i]) % nz
            fo = D.collide(po, f0[:, zs, ys, xs], site=(zs * ny + ys) * nx + xs, step=t)
            out[k, i] = fo[i]
    return out


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_256_cube_sampled_sites(flb, prec):
    """The 256^3 lattice the D3Q19 benchmark times (u0 = (0.1, 0, 0),
    kT = 1e-4, tau = 1 for all fifteen modes: the one-relaxation-time
    kernels), in FP32-shifted and FP64 storage: sampled sites (the eight
    corners and 64 random ones) recomputed one by one by the oracle from the
    GPU's own pre-step state, at both streaming phases.  FP64 to 1e-12 of
    max |f|; FP32 to 1e-5 of the largest fluctuation, the bar of the other
    FP32-shifted D3Q19 tests."""
    n = 256
    kw = dict(ux0=0.1, kT=1e-4, seed=1)
    precision = flb.FP64 if prec == "fp64" else flb.FP32_SHIFTED
    g = flb.Lattice3(flb.make_params3(n, n, n, precision=precision, **kw))
    po = D.make_params(n, n, n, **kw)
    rng = np.random.default_rng(4)
    sites = [(x, y, z) for x in (0, n - 1) for y in (0, n - 1) for z in (0, n - 1)]
    sites += [tuple(int(c) for c in rng.integers(0, n, 3)) for _ in range(64)]
    feq = D.equilibrium(1.0, 0.1, 0.0, 0.0)
    g.step(3)
    for _ in range(2):  # odd phase, then even phase
        t = g.t
        f0 = g.populations()
        g.step(1)
        f1 = g.populations()
        want = one_step_samples3(po, f0, t, sites, n, n, n)
        got = np.array([f1[:, z, y, x] for (x, y, z) in sites])
        del f0, f1
        err = np.abs(got - want).max()
        if prec == "fp64":
            rel = err / np.abs(want).max()
            bar = 1e-12
        else:
            rel = err / np.abs(want - feq).max()
            bar = 1e-5
        print(f"256^3 {prec} step {t}: max |f - oracle| = {err:.2e} ({rel:.2e} relative)")
        assert rel <= bar, (prec, t, err, rel)
