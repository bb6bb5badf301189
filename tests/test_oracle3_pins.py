"""Pins of the D3Q19 oracle (the generalisation the paper points to in
Sec. V; the model is described in oracle/flbref3.h) against what the
mathematics fixes: lattice symmetry and isotropy, orthonormality, the closed
forms of the conserved f-norm rows, a library Cholesky, the published
Philox bijection (through the D2Q9 oracle's own, itself pinned to rocRAND),
exact conservation, the BGK limit and the ideal-gas covariance at rest."""
import math

import numpy as np

import oracle as O
from oracle import d3q19 as D

VX, VY, VZ, W = D.velocities()
C = np.stack([VX, VY, VZ], axis=1).astype(float)


def polys():
    x, y, z = C.T
    x2, y2, z2 = x * x, y * y, z * z
    v2 = x2 + y2 + z2
    return np.array([np.ones(19), x, y, z, x * y, x * z, y * z, x2 - y2, x2 + y2 - 2 * z2, v2,
                     x * (y2 + z2), y * (x2 + z2), z * (x2 + y2), x * (y2 - z2), y * (z2 - x2),
                     z * (x2 - y2), v2 * v2, (2 * x2 - y2 - z2) * v2, (y2 - z2) * v2])


def test_velocity_set_symmetry_and_isotropy():
    assert len({tuple(c) for c in C}) == 19
    assert abs(W.sum() - 1) < 1e-15
    for i in range(1, 19):  # opposite pairs are adjacent
        j = i + 1 if i % 2 == 1 else i - 1
        assert (C[j] == -C[i]).all()
    d = np.eye(3)
    assert np.abs(np.einsum("i,ia,ib->ab", W, C, C) - d / 3).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib,ic->abc", W, C, C, C)).max() < 1e-15
    four = np.einsum("i,ia,ib,ic,id->abcd", W, C, C, C, C)
    want = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) +
            np.einsum("ad,bc->abcd", d, d)) / 9
    assert np.abs(four - want).max() < 1e-15


def test_basis_rows_are_the_gram_schmidt_of_the_polynomials():
    m = D.basis()
    assert np.abs(m @ np.diag(W) @ m.T - np.eye(19)).max() < 1e-13
    assert np.abs(m[0] - 1).max() < 1e-15
    for a, v in zip((1, 2, 3), (C[:, 0], C[:, 1], C[:, 2])):
        assert np.abs(m[a] - math.sqrt(3) * v).max() < 1e-14
    P = polys()
    for a in range(19):  # row a lies in span(P_0..P_a) with a positive P_a share
        coef, *_ = np.linalg.lstsq(P[:a + 1].T, m[a], rcond=None)
        assert np.abs(P[:a + 1].T @ coef - m[a]).max() < 1e-12
        assert coef[-1] > 0


def test_equilibrium_moments():
    rho, u = 1.2, np.array([0.1, -0.07, 0.04])
    f = D.equilibrium(rho, *u)
    assert abs(f.sum() - rho) < 1e-15
    assert np.abs(C.T @ f - rho * u).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib->ab", f, C, C) - rho * (np.outer(u, u) + np.eye(3) / 3)).max() < 1e-14


def test_fnorm_basis_orthonormal_closed_forms_and_cholesky():
    for u in [(0.0, 0.0, 0.0), (0.1, -0.05, 0.02), (0.2, 0.1, -0.15)]:
        mt = D.fnorm_basis(*u)
        g = D.equilibrium(1.0, *u)
        assert np.abs(mt @ np.diag(g) @ mt.T - np.eye(19)).max() < 1e-12
        assert np.abs(mt[0] - 1).max() < 1e-13
        for a in range(3):
            assert np.abs(mt[1 + a] - math.sqrt(3) * (C[:, a] - u[a])).max() < 1e-12
        m = D.basis()
        L = np.linalg.cholesky(m @ np.diag(g) @ m.T)  # library routine
        assert np.abs(mt - np.linalg.solve(L, m)).max() < 1e-11
    assert np.abs(D.fnorm_basis(0, 0, 0) - D.basis()).max() < 1e-13


def test_gaussian_draw_definition():
    """Four Philox blocks (counter word 1 = block index), top 24 bits,
    Box-Muller on consecutive pairs, as written in flbref3.h."""
    seed, site, step = 77, 1234, 5
    N = D.site_gaussians(seed, site, step)
    U = []
    for c in range(4):
        w = O.philox([site, c, step & 0xFFFFFFFF, step >> 32], [seed & 0xFFFFFFFF, seed >> 32])
        U += [int(x) >> 8 for x in w]
    want = []
    for p in range(8):
        ua, ub = (U[2 * p] + 0.5) / 2 ** 24, (U[2 * p + 1] + 0.5) / 2 ** 24
        r = math.sqrt(-2 * math.log(ua))
        want += [r * math.cos(2 * math.pi * ub), r * math.sin(2 * math.pi * ub)]
    assert np.abs(N - np.array(want[:15])).max() < 1e-15
    draws = np.array([D.site_gaussians(3, s, 11) for s in range(4000)]).ravel()
    assert abs(draws.mean()) < 0.03 and abs(draws.var() - 1) < 0.04


def test_collision_conserves_and_reduces_to_bgk():
    rng = np.random.default_rng(5)
    taus = rng.uniform(0.6, 1.5, 15)
    for basis in (D.BASIS_FNORM_LOCAL, D.BASIS_HERMITE):
        p = D.make_params(5, 5, 5, kT=1e-4, tau=taus, basis=basis)
        f = D.equilibrium(1.0, 0.1, -0.05, 0.03) * (1 + 0.01 * rng.standard_normal(19))
        fo = D.collide(p, f, site=17, step=3)
        assert abs(fo.sum() - f.sum()) < 1e-13
        assert np.abs(C.T @ (fo - f)).max() < 1e-13
        # noise-free, all tau equal: BGK towards f^0(rho, u) whatever the basis
        q = D.make_params(5, 5, 5, kT=0.0, tau=(0.8,), basis=basis)
        rho = f.sum()
        u = C.T @ f / rho
        want = f - (f - D.equilibrium(rho, *u)) / 0.8
        assert np.abs(D.collide(q, f) - want).max() < 1e-14
        feq = D.equilibrium(1.1, 0.05, 0.02, -0.04)
        assert np.abs(D.collide(q, feq) - feq).max() < 1e-15


def test_oracle_statistics_at_rest_match_closed_form():
    """3^3 lattice (odd sides: only the k = 0 mass and momentum are
    invariant), u0 = 0: <df_i df_j> = mu rho0 [w_i delta_ij - w_i w_j
    (1 + 3 v_i.v_j) / N] within standard errors."""
    n = 3
    kT = 1e-4
    p = D.make_params(n, n, n, kT=kT, seed=4, sample_every=1, block_steps=1000)
    L = D.Lattice(p)
    L.step(500)
    L.reset_stats()
    L.step(20000)
    c = L.covariance()
    N = n ** 3
    want = 3 * kT * (np.diag(W) - np.outer(W, W) * (1 + 3 * C @ C.T) / N)
    iu = np.triu_indices(19)
    z = ((c["cov_f"] - want) / c["se_cov_f"])[iu]
    zmax, zrms = np.abs(z).max(), math.sqrt((z ** 2).mean())
    assert zmax < 4.5 and 0.5 < zrms < 1.6, (zmax, zrms)
