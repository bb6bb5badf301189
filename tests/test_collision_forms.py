"""The algebra the step kernels use for the f-norm collision, pinned on the
CPU against the oracle's literal form (Sec. IV, eqs. (27)-(32); eq. (6)).

The oracle builds the f-norm rows m~ by Gram-Schmidt under <a,b>_g and adds
sum_a n~^a dM~^a with n~^a = m~^a g.  The kernels instead:
1. factor the Schur complement G' of the Hermite rows 3..8 under <,>_g
   (the projections on the conserved rows 1, sqrt3 (v - u) taken out) as
   G' = L L^T and take M~ = L^-1 d, d the Hermite non-equilibrium moments;
2. form the change as w_i sum_a m_i^a (L dM~)_a, the Hermite rows being
   orthonormal under the weights w: the change has no conserved moments and
   its Hermite moments on rows 3..8 are L dM~;
3. with one relaxation time, L dM~ = L (xi N) - d / tau (no solve).
These tests build (1)-(3) in numpy from the Hermite rows alone and check
them against the oracle's rows and its collision, to rounding; the same for
the nineteen rows of D3Q19."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import d3q19 as D

S3 = math.sqrt(3.0)


def rows():
    m = O.hermite_matrix()
    vx, vy, w = O.velocities()
    return m, np.asarray(vx, float), np.asarray(vy, float), w


def schur_factor(ux, uy):
    """L of G' = <m^a, m^b>_g - sum_c <c, m^a>_g <c, m^b>_g, a, b = 3..8,
    c over the conserved rows 1, sqrt3 (v_x - u_x), sqrt3 (v_y - u_y)."""
    m, vx, vy, _ = rows()
    g = O.equilibrium(1.0, ux, uy)
    cons = np.stack([np.ones(9), S3 * (vx - ux), S3 * (vy - uy)])
    hm = m[3:]
    G = hm @ np.diag(g) @ hm.T
    P = cons @ np.diag(g) @ hm.T
    return np.linalg.cholesky(G - P.T @ P)


@pytest.mark.parametrize("ux,uy", [(0.0, 0.0), (0.1, -0.05), (0.3, 0.2), (-0.25, 0.35)])
def test_change_through_hermite_rows_equals_the_fnorm_sum(ux, uy):
    """For random dM~, sum_a n~^a dM~^a with the oracle's Gram-Schmidt rows
    has no conserved Hermite moments, its moments on rows 3..8 are L dM~,
    and it equals w_i sum_a m_i^a (L dM~)_a."""
    m, _, _, w = rows()
    mt = O.fnorm_basis(ux, uy)  # the oracle's rows m~ (Gram-Schmidt under g)
    g = O.equilibrium(1.0, ux, uy)
    L = schur_factor(ux, uy)
    rng = np.random.default_rng(7)
    for _ in range(20):
        dM = rng.standard_normal(6)
        df = (mt[3:] * g).T @ dM  # sum_a m~^a g dM~^a
        assert np.abs(m[:3] @ df).max() < 1e-14
        np.testing.assert_allclose(m[3:] @ df, L @ dM, rtol=0, atol=1e-13)
        np.testing.assert_allclose(df, w * (m[3:].T @ (L @ dM)), rtol=0, atol=1e-14)


@pytest.mark.parametrize("ux,uy", [(0.1, -0.05), (0.3, 0.2)])
def test_forward_solve_gives_the_fnorm_moments(ux, uy):
    """M~^{3..8} = <m~^a, f - f^0(rho, u)> equals L^-1 d."""
    m, _, _, _ = rows()
    mt = O.fnorm_basis(ux, uy)
    L = schur_factor(ux, uy)
    rng = np.random.default_rng(3)
    feq = O.equilibrium(1.0, ux, uy)
    for _ in range(10):
        # a state with the same rho and u: change only non-conserved moments
        df = (O.fnorm_basis(ux, uy)[3:] * feq).T @ (1e-3 * rng.standard_normal(6))
        f = feq + df
        d = m[3:] @ (f - feq)
        np.testing.assert_allclose(np.linalg.solve(L, d), mt[3:] @ (f - feq), rtol=0,
                                   atol=1e-15)


def kernel_form(f, tau, kT, gauss, one_tau):
    """The collision as the kernels compute it (FP64, numpy)."""
    m, vx, vy, w = rows()
    rho = f.sum()
    ux, uy = (m[1] @ f) / (S3 * rho), (m[2] @ f) / (S3 * rho)
    d = m[3:] @ (f - O.equilibrium(rho, ux, uy))
    L = schur_factor(ux, uy)
    tau = np.asarray(tau, float)
    xi = np.sqrt(3.0 * kT * rho * (2.0 * tau - 1.0)) / tau
    if one_tau:
        Y = L @ (xi * gauss) - d / tau[0]
    else:
        Y = L @ (xi * gauss - np.linalg.solve(L, d) / tau)
    return f + w * (m[3:].T @ Y)


@pytest.mark.parametrize("tau,one_tau", [((0.8,) * 6, True), ((0.8,) * 6, False),
                                         ((0.6, 0.9, 1.2, 0.7, 1.5, 1.0), False)])
@pytest.mark.parametrize("ux0,uy0", [(0.0, 0.0), (0.1, -0.05), (0.3, 0.2)])
def test_kernel_form_equals_the_oracle_collision(tau, one_tau, ux0, uy0):
    """The whole collision of a perturbed state, with noise, in the kernels'
    form (general, and with one relaxation time the form without the solve)
    against the oracle's collision of the same site and step."""
    kT, seed = 1e-3, 11
    p = O.make_params(4, 4, ux0=ux0, uy0=uy0, kT=kT, tau=tau, seed=seed)
    rng = np.random.default_rng(5)
    for site, step in ((0, 0), (5, 3), (13, 1000)):
        f = O.equilibrium(1.0 + 0.01 * rng.standard_normal(), ux0 + 0.01 * rng.standard_normal(),
                          uy0 + 0.01 * rng.standard_normal())
        f = f + 1e-4 * rng.standard_normal(9)
        want = O.collide(p, f, site=site, step=step)
        got = kernel_form(f, tau, kT, O.site_gaussians(seed, site, step), one_tau)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


# ------------------------------------------------------------------ D3Q19
# The same algebra with nineteen rows: four conserved (1, sqrt3 (v_a - u_a))
# and fifteen relaxed (the D3Q19 generalisation of Sec. V).


def schur_factor3(u):
    m = D.basis()
    vx, vy, vz, _ = D.velocities()
    v = np.stack([vx, vy, vz]).astype(float)
    g = D.equilibrium(1.0, *u)
    cons = np.vstack([np.ones(19)] + [S3 * (v[a] - u[a]) for a in range(3)])
    hm = m[4:]
    G = hm @ np.diag(g) @ hm.T
    P = cons @ np.diag(g) @ hm.T
    return np.linalg.cholesky(G - P.T @ P)


@pytest.mark.parametrize("u", [(0.0, 0.0, 0.0), (0.1, -0.05, 0.03), (0.2, 0.1, -0.15)])
def test_d3q19_change_through_hermite_rows_equals_the_fnorm_sum(u):
    m = D.basis()
    w = D.velocities()[3]
    mt = D.fnorm_basis(*u)
    g = D.equilibrium(1.0, *u)
    L = schur_factor3(u)
    rng = np.random.default_rng(8)
    for _ in range(10):
        dM = rng.standard_normal(15)
        df = (mt[4:] * g).T @ dM
        assert np.abs(m[:4] @ df).max() < 1e-13
        np.testing.assert_allclose(m[4:] @ df, L @ dM, rtol=0, atol=1e-12)
        np.testing.assert_allclose(df, w * (m[4:].T @ (L @ dM)), rtol=0, atol=1e-13)


@pytest.mark.parametrize("one_tau", [True, False])
def test_d3q19_kernel_form_equals_the_oracle_collision(one_tau):
    """The D3Q19 f-norm collision with noise in the kernels' form (Y seeded
    with -d / tau and L (xi N) added for one relaxation time; L (xi N -
    L^-1 d / tau) otherwise) against the oracle's collision."""
    m = D.basis()
    w = D.velocities()[3]
    if one_tau:
        tau = np.full(15, 0.8)
    else:
        tau = np.round(np.random.default_rng(2).uniform(0.6, 1.5, 15), 6)
    kT, seed, u0 = 1e-3, 9, (0.1, -0.05, 0.03)
    p = D.make_params(3, 3, 3, ux0=u0[0], uy0=u0[1], uz0=u0[2], kT=kT, tau=tuple(tau), seed=seed)
    rng = np.random.default_rng(6)
    for site, step in ((0, 0), (7, 2), (26, 999)):
        f = D.equilibrium(1.0 + 0.01 * rng.standard_normal(),
                          *(u0[a] + 0.01 * rng.standard_normal() for a in range(3)))
        f = f + 1e-4 * rng.standard_normal(19)
        want = D.collide(p, f, site=site, step=step)
        rho = f.sum()
        u = (m[1:4] @ f) / (S3 * rho)
        d = m[4:] @ (f - D.equilibrium(rho, *u))
        L = schur_factor3(u)
        xi = np.sqrt(3.0 * kT * rho * (2.0 * tau - 1.0)) / tau
        N = D.site_gaussians(seed, site, step)
        if one_tau:
            Y = -d / tau[0] + L @ (xi * N)
        else:
            Y = L @ (xi * N - np.linalg.solve(L, d) / tau)
        got = f + w * (m[4:].T @ Y)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)
