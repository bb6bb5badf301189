"""Linear-response prediction of the equal-time fluctuation statistics.

Test infrastructure only (imported by tests and by nothing in the product).

Sec. II linearises the fluctuating update around the mean state
<f_i> = f_i^0(rho0, u0) (eqs. (7)-(10)), Fourier transforms it in space and
follows the covariance of the fluctuations through one update (eqs. (11)-(14)).
The paper then keeps only k = 0 and stationarity to derive its FDT (eq. (15)).
Here the same recursion is solved for every wavevector on the lattice:

    df(k, t+1) = S(k) [ A df(k, t) + eta(k, t) ],
    S(k) = diag(exp(-i k.v_i))               (streaming, eq. (1)),
    A    = d f* / d f at f^0(rho0, u0)        (noise-free collision),
    <eta eta^T> = Q = sum_{a>=3} xi_a^2 n~^a n~^a^T   (eqs. (6), (20)),

so the stationary covariance c(k) = <df(k) df(k)^H> (unitary transform)
solves the discrete Lyapunov equation c = T c T^H + S Q S^H with T = S A.
The equal-time, same-site covariance is (1/(nx ny)) sum_k c(k), and the
structure factor of a measured field B.df is B c(k) B^H.

At wavevectors where T has a unit-modulus eigenvalue (k = 0 with the exact
invariants rho, j_x, j_y; for an even side also the staggered j_x at
(pi, 0) and j_y at (0, pi)) the equation is singular; there the
covariance is summed from c = 0 by repeated doubling, which leaves the
invariant directions at their initial (zero) fluctuation.

The collision Jacobian is taken by central differences of the oracle's
own noise-free collision; the noise matrix uses the basis construction of
the oracle at (rho0, u0).
"""
from __future__ import annotations

import numpy as np

import oracle as O


def noise_strength(kT: float) -> float:
    """mu = kT / theta with theta = 1/3 (Sec. II, eq. (20), scaled)."""
    return kT * 3.0


def jacobian(p: "O.Params", h: float = 1e-5) -> np.ndarray:
    """A_ij = d f*_i / d f_j of the noise-free collision at f^0(rho0, u0).

    Fourth-order central differences of the oracle's collision; the result
    is then corrected by an O(rounding) oblique projection so that the
    collision conserves mass and momentum exactly (c^T (A - I) = 0 for
    c = 1, v_x, v_y).  Without it the exact invariants of the lattice become
    nearly-invariant and the singular wavevectors pick up spurious weight."""
    q = O.make_params(p.nx, p.ny, rho0=p.rho0, ux0=p.ux0, uy0=p.uy0, kT=0.0,
                      tau=list(p.tau), basis=p.basis)
    f0 = O.equilibrium(p.rho0, p.ux0, p.uy0)
    A = np.zeros((9, 9))
    d = h * p.rho0
    for j in range(9):
        e = np.zeros(9)
        e[j] = d
        A[:, j] = (-O.collide(q, f0 + 2 * e) + 8 * O.collide(q, f0 + e)
                   - 8 * O.collide(q, f0 - e) + O.collide(q, f0 - 2 * e)) / (12 * d)
    vx, vy, _ = O.velocities()
    Cm = np.stack([np.ones(9), vx, vy], axis=1).astype(float)  # 9 x 3
    Wg = np.diag(f0 / p.rho0)
    D = A - np.eye(9)
    D -= Wg @ Cm @ np.linalg.solve(Cm.T @ Wg @ Cm, Cm.T @ D)
    return np.eye(9) + D


def noise_matrix(p: "O.Params") -> np.ndarray:
    """Q = sum_{a>=3} xi_a^2 n~^a n~^a^T at (rho0, u0)."""
    mu = noise_strength(p.kT)
    if p.basis == O.BASIS_HERMITE:
        _, _, w = O.velocities()
        mt = O.hermite_matrix()
        nt = mt * w[None, :]
    elif p.basis == O.BASIS_FNORM_LUT:
        mt, ug = O.lut_basis(p.ux0, p.uy0)
        nt = mt * O.equilibrium(1.0, ug[0], ug[1])[None, :]
    else:
        mt = O.fnorm_basis(p.ux0, p.uy0)
        nt = mt * O.equilibrium(1.0, p.ux0, p.uy0)[None, :]
    Q = np.zeros((9, 9))
    for a in range(3, 9):
        tau = p.tau[a - 3]
        xi2 = mu * p.rho0 * (2 * tau - 1) / tau ** 2
        Q += xi2 * np.outer(nt[a], nt[a])
    return Q


def _doubling(T: np.ndarray, Q: np.ndarray, n: int = 24) -> np.ndarray:
    c = Q.copy()
    Tn = T.copy()
    for _ in range(n):
        c = c + Tn @ c @ Tn.conj().T
        Tn = Tn @ Tn
    return c


def k_covariances_at(p: "O.Params", kx_idx, ky_idx, A: np.ndarray | None = None,
                     Q: np.ndarray | None = None) -> np.ndarray:
    """c(k) at the wavevectors k = 2 pi (kx_idx / nx, ky_idx / ny) (integer
    index arrays of one shape), shape (..., 9, 9)."""
    vx, vy, _ = O.velocities()
    A = jacobian(p) if A is None else A
    Q = noise_matrix(p) if Q is None else Q
    KX = 2 * np.pi * np.asarray(kx_idx, dtype=float) / p.nx
    KY = 2 * np.pi * np.asarray(ky_idx, dtype=float) / p.ny
    shape = KX.shape
    ph = np.exp(-1j * (KX.reshape(-1)[:, None] * vx + KY.reshape(-1)[:, None] * vy))  # (n, 9)
    T = ph[:, :, None] * A[None, :, :]
    Qk = ph[:, :, None] * Q[None] * ph.conj()[:, None, :]
    out = np.zeros((len(ph), 9, 9), dtype=complex)
    eig = np.abs(np.linalg.eigvals(T)).max(axis=-1)
    singular = eig > 1 - 1e-9
    # regular wavevectors: vec(c) = (I - conj(T) (x) T)^-1 vec(Q) (row-major vec)
    reg = np.flatnonzero(~singular)
    eye = np.eye(81)
    for start in range(0, len(reg), 4096):
        idx = reg[start:start + 4096]
        Tb = T[idx]
        K = np.einsum("nij,nkl->nikjl", Tb, Tb.conj()).reshape(-1, 81, 81)
        sol = np.linalg.solve(eye[None] - K, Qk[idx].reshape(-1, 81, 1))
        out[idx] = sol.reshape(-1, 9, 9)
    for n in np.flatnonzero(singular):
        out[n] = _doubling(T[n], Qk[n])
    return out.reshape(*shape, 9, 9)


def k_covariances(p: "O.Params", A: np.ndarray | None = None, Q: np.ndarray | None = None):
    """c(k) for every lattice wavevector, shape (ny, nx, 9, 9), index [ky, kx]."""
    KX, KY = np.meshgrid(np.arange(p.nx), np.arange(p.ny))  # [ky, kx]
    return k_covariances_at(p, KX, KY, A, Q)


def site_covariance(p: "O.Params", ck=None) -> np.ndarray:
    """<df_i df_j> at one site: the mean of c(k) over the Brillouin zone."""
    ck = k_covariances(p) if ck is None else ck
    return ck.reshape(-1, 9, 9).mean(axis=0).real


def ideal_covariance_u0_zero(p: "O.Params") -> np.ndarray:
    """Closed form at u0 = 0: mu rho0 [w_i delta_ij - w_i w_j (1 + c v_i.v_j) / (nx ny)],
    c = 3 for odd sides (the k = 0 invariants rho, j_x, j_y removed) and
    c = 6 when both sides are even (the staggered j_x, j_y invariants at
    (pi,0), (0,pi) removed as well).  Eq. (16) with the invariant modes of
    the finite periodic lattice taken out."""
    vx, vy, w = O.velocities()
    mu = noise_strength(p.kT)
    vv = np.outer(vx, vx) + np.outer(vy, vy)
    extra = np.zeros((9, 9))
    if p.nx % 2 == 0:
        extra += 3 * np.outer(vx, vx)
    if p.ny % 2 == 0:
        extra += 3 * np.outer(vy, vy)
    corr = np.outer(w, w) * (1 + 3 * vv + extra)
    return mu * p.rho0 * (np.diag(w) - corr / (p.nx * p.ny))


def moment_covariance(p: "O.Params", C: np.ndarray, basis: str = "fnorm_u0") -> np.ndarray:
    """B C B^T with B the f-norm basis at u0 (Sec. IV measurement) or Hermite."""
    B = O.fnorm_basis(p.ux0, p.uy0) if basis == "fnorm_u0" else O.hermite_matrix()
    return B @ C @ B.T


def structure_factors(p: "O.Params", ck=None) -> dict:
    """Predicted <|dA(k)|^2>/(nx ny) for rho, j~_x, j~_y at u0 and the cross term
    (for every wavevector, or for the c(k) given)."""
    ck = k_covariances(p) if ck is None else ck
    B = O.fnorm_basis(p.ux0, p.uy0)
    b0 = np.ones(9)
    b1, b2 = B[1], B[2]
    s = lambda u, v: np.einsum("i,...ij,j->...", u, ck, v)
    x12 = s(b1, b2)
    return {"rho": s(b0, b0).real, "jx": s(b1, b1).real, "jy": s(b2, b2).real,
            "jxjy_re": x12.real, "jxjy_im": x12.imag}


def fit_lq(us, values):
    """Least-squares fit of values(u) = l u + q u^2 (no constant), as in
    Figs. 7 and 18."""
    us = np.asarray(us, dtype=float)
    X = np.stack([us, us ** 2], axis=1)
    coef, *_ = np.linalg.lstsq(X, np.asarray(values, dtype=float), rcond=None)
    return coef[0], coef[1]


# Bands of wavevectors for averaging structure factors: |m| in [lo, hi) with
# m = (mx, my) the integer wavevector taken in [-n/2, n/2); "axis" bands
# keep only my = 0 (the cut along k_x of the paper's figures).  The k = 0
# mode and, for even sides, the staggered (n/2, 0) and (0, n/2) modes (exact
# invariants, never excited) are left out, and so is |m| < 2: on a 256-wide
# lattice those hydrodynamic modes decorrelate over ~5000 steps, too slowly
# for errors from blocks of that length.
PLANE_EDGES = (2, 4, 8, 16, 32, 64, 128, 200)
AXIS_EDGES = (2, 4, 16, 64, 129)


def band_masks(nx: int, ny: int, edges=PLANE_EDGES, axis: bool = False):
    """Boolean masks [ky, kx], one per band."""
    mx = np.fft.fftfreq(nx, 1.0 / nx)
    my = np.fft.fftfreq(ny, 1.0 / ny)
    MX, MY = np.meshgrid(mx, my)
    r = np.hypot(MX, MY)
    keep = r > 0
    if nx % 2 == 0:
        keep &= ~((np.abs(MX) == nx // 2) & (MY == 0))
    if ny % 2 == 0:
        keep &= ~((MX == 0) & (np.abs(MY) == ny // 2))
    if axis:
        keep &= MY == 0
    return [keep & (r >= lo) & (r < hi) for lo, hi in zip(edges[:-1], edges[1:])]


def band_means(S: np.ndarray, masks) -> np.ndarray:
    """Mean of S[ky, kx] over each band."""
    return np.array([S[m].mean() for m in masks])
