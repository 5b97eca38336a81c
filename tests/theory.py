"""Closed forms used by the statistical and deterministic checks (test side).

Lattice symbols: Shinozaki-Oono Laplacian (the paper's Eq. solapft in 3-D, its
2-D analogue), FV Gamma and Gamma.Gamma for D2Q9/D3Q15/D3Q19 (for D3Q15 the
paper's own Eq. fvlapft), central difference.
SMOL discrete-time response for frozen-noise Runge-Kutta: the stability
polynomial R(z) and noise transfer phi(z), the static structure factor
2 kT M (-L_out) |phi|^2 / (1 - |R|^2), whose dt -> 0 limit is kT/(A - K L_SO)
(Eq. test2 and the text after it).
"""
import numpy as np

D2Q9, D3Q15, D3Q19 = 9, 15, 19
FD, FV = 0, 1


def so_symbol(q, lattice):
    c = np.cos(q)
    if lattice != D2Q9:
        return (12 * (c[0] + c[1] + c[2]) + 12 * (c[0] * c[1] + c[0] * c[2] + c[1] * c[2])
                + 8 * c[0] * c[1] * c[2] - 80) / 22
    return c[0] + c[1] + c[0] * c[1] - 3


def fv_gamma(q, lattice):
    """Imaginary part of the FV gradient symbol Gamma(q) (Gamma = i * this)."""
    s, c = np.sin(q), np.cos(q)
    if lattice == D3Q19:
        return np.array([s[0] * (1 + c[1] + c[2]), s[1] * (1 + c[0] + c[2]),
                         s[2] * (1 + c[0] + c[1])]) / 3
    if lattice == D3Q15:
        return np.array([s[0] * (2 + c[1] * c[2]), s[1] * (2 + c[0] * c[2]),
                         s[2] * (2 + c[0] * c[1])]) / 3
    return np.array([s[0] * (2 + c[1]), s[1] * (2 + c[0])]) / 3


def l_out(q, lattice, smol):
    if smol == FD:
        return so_symbol(q, lattice)
    g = fv_gamma(q, lattice)
    return -(g * g).sum(axis=0)


def advection_symbol(q, U, lattice, smol):
    """theta with -Div(U psi) -> -i theta psi."""
    d = 2 if lattice == D2Q9 else 3
    U = np.asarray(U, dtype=float)[:d]
    if smol == FD:
        s = np.sin(q[:d])
    else:
        s = fv_gamma(q, lattice)
    return np.tensordot(U, s, axes=(0, 0))


def rk_poly(z, stages):
    if stages == 1:
        return 1 + z, np.ones_like(z)
    if stages == 2:
        return 1 + z + z * z / 2, 1 + z / 2
    return (1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24,
            1 + z / 2 + z ** 2 / 6 + z ** 3 / 24)


def smol_z(q, lattice, smol, M, a, kappa, U=(0, 0, 0)):
    lso = so_symbol(q, lattice)
    lo = l_out(q, lattice, smol)
    lam = M * (-lo) * (a - kappa * lso)
    return -lam - 1j * advection_symbol(q, U, lattice, smol), lo, lso


def smol_static_sk(q, lattice, smol, M, a, kappa, kT, stages=2, U=(0, 0, 0)):
    z, lo, lso = smol_z(q, lattice, smol, M, a, kappa, U)
    R, phi = rk_poly(z, stages)
    with np.errstate(divide="ignore", invalid="ignore"):
        return 2 * kT * M * (-lo) * np.abs(phi) ** 2 / (1 - np.abs(R) ** 2)


def ornstein_zernike(q, lattice, a, kappa, kT):
    return kT / (a - kappa * so_symbol(q, lattice))


def axis_q(L, axis, d):
    """Wave vectors 2 pi m / L along one axis, as a (3, L) array."""
    q = np.zeros((3, L))
    q[axis] = 2 * np.pi * np.arange(L) / L
    return q


def n_eff(decay, nsamp, every):
    """Effectively independent samples of |X_q|^2 for a mode whose amplitude
    decays by the factor `decay` per step (|R| for psi, exp(-rate) for the
    fluid), sampled `nsamp` times every `every` steps: the correlation of
    |X_q|^2 between samples is decay^(2 every), and the variance of the mean
    of an AR(1) series with that coefficient is that of
    nsamp (1 - rho)/(1 + rho) independent samples."""
    with np.errstate(invalid="ignore", over="ignore"):
        rho = np.clip(decay, 0, 1) ** (2 * every)
        return np.maximum(nsamp * (1 - rho) / (1 + rho), 1.0)


def mean_and_se(ratios, neff):
    """Mean of per-mode ratios <|X_q|^2>/theory over independent modes, and
    its standard error: |X_q|^2 of a Gaussian mode has relative variance 1 per
    independent sample, so each ratio carries variance 1/n_eff."""
    ratios = np.asarray(ratios, dtype=float)
    neff = np.asarray(neff, dtype=float)
    return ratios.mean(), np.sqrt((1.0 / neff).sum()) / ratios.size


def axis_modes(L):
    """Independent axis wave numbers of a real field: m = 1 .. L/2 (m and L-m
    are one mode)."""
    return np.arange(1, L // 2 + 1)


def interp_gain(delta, l):
    """Gain d h_est / d h of the linear-interpolation height estimator
    (Sec. VI.C) on the tanh profile psi = psi_eq tanh((z - h)/l) of Eq. (tanh),
    for an interface at fractional offset delta in [0, 1) above the site z0:
    h_est - z0 = t(delta)/(t(delta) + t(1 - delta)), t(x) = tanh(x/l).  It is
    1/(l tanh(1/l)) > 1 with the interface on a site, below 1 half-way between
    sites, and its mean over the offsets is exactly 1 (h_est runs from z0 to
    z0 + 1 as delta does)."""
    a = np.tanh(np.asarray(delta, dtype=float) / l)
    b = np.tanh((1.0 - np.asarray(delta, dtype=float)) / l)
    da = (1.0 - a * a) / l
    db = -(1.0 - b * b) / l
    return (da * b - a * db) / (a + b) ** 2


def height_gain(h, l):
    """Long-wavelength gain of the height estimator over the columns of one
    snapshot: the mean of interp_gain over the columns' offsets.  Where the
    roughness is below a lattice spacing every column has the same offset and
    the gain is that column's; a rough interface samples all offsets and the
    gain tends to 1."""
    h = np.asarray(h, dtype=float)
    return float(np.mean(interp_gain(h - np.floor(h), l)))


def smol_linear_operators(p):
    """Matrices of the oracle's SMOL with B = 0 and no flow: the right-hand
    side L (G(phi) = L phi + N), the free-energy Hessian H = A - K L_SO and
    the divergence Dv that maps node noise to N, each built column by column
    from unit fields (so they carry whatever boundary rules the oracle has)."""
    import oracle as O
    N, d = O.nsites(p), O.d_of(p)
    L = np.zeros((N, N))
    H = np.zeros((N, N))
    Dv = np.zeros((N, d * N))
    zu, zn = np.zeros((d, N)), np.zeros(N)
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        L[:, k] = O.smol_rhs(p, e, zu, zn)
        H[:, k] = p.a * e - p.kappa * O.laplacian(p, e)
    for k in range(d * N):
        e = np.zeros(d * N)
        e[k] = 1.0
        Dv[:, k] = O.divergence(p, e.reshape(d, N))
    return L, H, Dv


def stationary_covariance(L, H, Dv, kT, M, stages=2):
    """Stationary covariance of psi - mean(psi) under the frozen-noise
    Runge-Kutta step psi' = R(L) psi + Phi(L) N, N of covariance
    2 kT M Dv Dv^T (the node noise of amplitude sqrt(2 kT M)), with R and Phi
    the stage polynomials of rk_poly.  It solves C = R C R^T + Phi S Phi^T.
    With L = M Dv Grad H, H symmetric positive definite and Dv Grad
    symmetric, L is symmetric in the metric of H: in the basis
    H^(1/2) (eigenvectors U of H^(1/2) L H^(-1/2)) the equation is diagonal,
    C'_ij = Q'_ij / (1 - r_i r_j); the conserved uniform mode (r = 1) carries
    no noise and is left out."""
    w, V = np.linalg.eigh((H + H.T) / 2)
    S = V @ np.diag(np.sqrt(w)) @ V.T
    Si = V @ np.diag(1 / np.sqrt(w)) @ V.T
    Lh = S @ L @ Si
    lam, U = np.linalg.eigh((Lh + Lh.T) / 2)
    r, ph = rk_poly(lam, stages)
    Q = U.T @ S @ (2 * kT * M * Dv @ Dv.T) @ S @ U
    Q = ph[:, None] * Q * ph[None, :]
    den = 1 - r[:, None] * r[None, :]
    cons = np.abs(lam) < 1e-12 * np.abs(lam).max()
    C = np.where(cons[:, None] | cons[None, :], 0.0, Q / np.where(cons[:, None] | cons[None, :],
                                                                   1.0, den))
    return Si @ U @ C @ U.T @ Si
