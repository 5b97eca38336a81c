"""Pins of the oracle's SMOL update (Sec. V) and of its noise law.

* Deterministic closed form (kT = 0, B = 0, imposed uniform flow U): a single
  Fourier mode is multiplied each step by the Runge-Kutta stability polynomial
  R(z) of the scheme, z = -lambda - i theta, with lambda = M (-L_out)(A - K L_SO)
  and theta the advection symbol U.s(q).  This pins the diffusion operator, the
  advection normalisation (FV reading) and the stage arithmetic (Euler, Heun, RK4).
* FDT at the lattice level (Sec. III): the covariance of the conserved noise
  equals -2 kT M times the diffusion operator L_out (FD: link fluxes against the
  Shinozaki-Oono Laplacian; FV: Gamma.xi against Gamma.Gamma), checked by brute
  force on small lattices.
"""
import numpy as np
import pytest

import oracle as O

CASES = [(O.D2Q9, (10, 8, 1)), (O.D3Q15, (5, 6, 4)), (O.D3Q19, (6, 5, 4))]


def _coords(p):
    N = O.nsites(p)
    s = np.arange(N)
    return np.stack([s % p.nx, (s // p.nx) % p.ny, s // (p.nx * p.ny)])


def _so_symbol(q, lattice):
    c = np.cos(q)
    if lattice != O.D2Q9:
        return (12 * c.sum() + 12 * (c[0] * c[1] + c[0] * c[2] + c[1] * c[2])
                + 8 * c.prod() - 80) / 22
    return c[0] + c[1] + c[0] * c[1] - 3


def _fv_gamma(q, lattice):
    s, c = np.sin(q), np.cos(q)
    if lattice == O.D3Q19:
        return np.array([s[0] * (1 + c[1] + c[2]), s[1] * (1 + c[0] + c[2]),
                         s[2] * (1 + c[0] + c[1])]) / 3
    if lattice == O.D3Q15:
        return np.array([s[0] * (2 + c[1] * c[2]), s[1] * (2 + c[0] * c[2]),
                         s[2] * (2 + c[0] * c[1])]) / 3
    return np.array([s[0] * (2 + c[1]), s[1] * (2 + c[0])]) / 3


def _R(z, stages):
    if stages == 1:
        return 1 + z
    if stages == 2:
        return 1 + z + z * z / 2
    return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24


@pytest.mark.parametrize("lattice,shape", CASES)
@pytest.mark.parametrize("smol", [O.FD, O.FV])
@pytest.mark.parametrize("stages", [1, 2, 4])
def test_single_mode_closed_form(lattice, shape, smol, stages):
    d = 2 if lattice == O.D2Q9 else 3
    U = np.array([0.05, -0.03, 0.02])[:d]
    p = O.make_params(lattice=lattice, smol=smol, coupling=O.SMOL_ONLY, rk_stages=stages,
                      shape=shape, kT=0.0, b=0.0, a=0.06, kappa=0.04, M=0.1,
                      u_imposed=tuple(U) + (0,) * (3 - d))
    X = _coords(p)[:d]
    L = np.array([p.nx, p.ny, p.nz])[:d]
    for k in [(1, 0, 0), (2, 3, 1), (L[0] // 2, 1, 2), (1, L[1] - 1, 1)]:
        q = 2 * np.pi * np.array(k[:d]) / L
        wave = np.exp(1j * (q @ X))
        lso = _so_symbol(q, lattice)
        if smol == O.FD:
            lout = lso
            theta = U @ np.sin(q)
        else:
            g = _fv_gamma(q, lattice)
            lout = -(g @ g)
            theta = U @ g
        lam = p.M * (-lout) * (p.a - p.kappa * lso)
        z = -lam - 1j * theta
        f0, _ = O.init(p)
        nsteps = 7
        for part in (np.real, np.imag):
            psi = np.ascontiguousarray(part(wave))
            f = f0.copy()
            O.run(p, f, psi, 0, nsteps)
            expect = part(_R(z, stages) ** nsteps * wave)
            np.testing.assert_allclose(psi, expect, atol=1e-13)
            np.testing.assert_array_equal(f, f0)  # SMOL_ONLY leaves the fluid alone


def _matrix(fn, n_in, n_out):
    M = np.zeros((n_out, n_in))
    for j in range(n_in):
        e = np.zeros(n_in)
        e[j] = 1.0
        M[:, j] = fn(e).reshape(-1)
    return M


@pytest.mark.parametrize("lattice,shape", [(O.D2Q9, (5, 4, 1)), (O.D3Q15, (4, 4, 3)),
                                           (O.D3Q19, (4, 4, 3))])
def test_fd_link_noise_covariance(lattice, shape):
    p = O.make_params(lattice=lattice, smol=O.FD, shape=shape, kT=0.7, M=0.3)
    N = O.nsites(p)
    nl = len(O.links(lattice)[1])
    E = _matrix(lambda z: O.fd_noise_divergence(p, z.reshape(nl, N)), nl * N, N)
    Lso = _matrix(lambda v: O.laplacian(p, v), N, N)
    np.testing.assert_allclose(E @ E.T, -2 * p.kT * p.M * Lso, atol=1e-14)
    # The noise is a divergence: it conserves psi exactly.
    np.testing.assert_allclose(E.sum(axis=0), 0.0, atol=1e-14)


@pytest.mark.parametrize("lattice,shape", [(O.D2Q9, (6, 5, 1)), (O.D3Q15, (4, 3, 5)),
                                           (O.D3Q19, (5, 4, 3))])
def test_fd_fourier_noise_covariance(lattice, shape):
    """The literal Fourier-space FD noise of Sec. V.A (Eq. etafdt): the linear
    map K from the white field to N must have covariance K K^T = -2 kT M L_SO
    with L_SO the oracle's real-space stencil, be symmetric, and conserve psi.
    Non-cubic sides catch transposed axes; a missing square root, scale or
    sign of the transform breaks the covariance."""
    p = O.make_params(lattice=lattice, smol=O.FD, shape=shape, kT=0.7, M=0.3,
                      fd_noise=O.FDNOISE_FOURIER)
    N = O.nsites(p)
    K = _matrix(lambda w: O.fd_noise_fourier(p, w), N, N)
    Lso = _matrix(lambda v: O.laplacian(p, v), N, N)
    np.testing.assert_allclose(K @ K.T, -2 * p.kT * p.M * Lso, atol=1e-13)
    np.testing.assert_allclose(K, K.T, atol=1e-14)
    np.testing.assert_allclose(K.sum(axis=0), 0.0, atol=1e-13)


def test_fd_fourier_noise_drives_the_step():
    """With fd_noise = Fourier the step's N^n is the Fourier map applied to the
    white field of normal slot 0 (same Philox stream as the link fluxes)."""
    p = O.make_params(lattice=O.D2Q9, smol=O.FD, shape=(7, 6, 1), kT=0.2, M=0.3,
                      fd_noise=O.FDNOISE_FOURIER)
    N = O.nsites(p)
    w = np.array([O.normal(p.seed, s, 11, O.TAG_SMOL, 0) for s in range(N)])
    np.testing.assert_allclose(O.smol_noise(p, 11), O.fd_noise_fourier(p, w), atol=1e-15)
    p_link = O.make_params(lattice=O.D2Q9, smol=O.FD, shape=(7, 6, 1), kT=0.2, M=0.3)
    assert np.abs(O.smol_noise(p_link, 11) - O.smol_noise(p, 11)).max() > 1e-3


@pytest.mark.parametrize("lattice,shape", [(O.D2Q9, (5, 4, 1)), (O.D3Q15, (4, 4, 3)),
                                           (O.D3Q19, (4, 4, 3))])
def test_fv_noise_covariance(lattice, shape):
    p = O.make_params(lattice=lattice, smol=O.FV, shape=shape, kT=0.7, M=0.3)
    N = O.nsites(p)
    d = O.d_of(p)
    Div = _matrix(lambda v: O.divergence(p, v.reshape(d, N)), d * N, N)
    Grad = _matrix(lambda v: O.gradient(p, v), N, d * N)
    Lfv = Div @ Grad
    cov = 2 * p.kT * p.M * Div @ Div.T
    np.testing.assert_allclose(cov, -2 * p.kT * p.M * Lfv, atol=1e-14)
    np.testing.assert_allclose(Grad, -Div.T, atol=1e-15)  # summation by parts


@pytest.mark.parametrize("lattice,shape,smol", [(O.D2Q9, (16, 12, 1), O.FD),
                                                (O.D2Q9, (16, 12, 1), O.FV),
                                                (O.D3Q19, (6, 6, 6), O.FD),
                                                (O.D3Q19, (6, 6, 6), O.FV),
                                                (O.D3Q15, (6, 6, 6), O.FV)])
def test_generated_noise_variance(lattice, shape, smol):
    # Realised noise (Philox) has the diagonal variance -2 kT M L_out(0 offset).
    p = O.make_params(lattice=lattice, smol=smol, shape=shape, kT=2.0, M=0.25)
    N = O.nsites(p)
    samples = np.array([O.smol_noise(p, n) for n in range(300)])
    if smol == O.FD:
        diag = -O.laplacian(p, np.eye(N)[0])[0]
    else:
        d = O.d_of(p)
        diag = -O.divergence(p, O.gradient(p, np.eye(N)[0]))[0]
    var = samples.var()
    expect = 2 * p.kT * p.M * diag
    assert abs(var / expect - 1) < 5 * np.sqrt(2 / samples.size) * 3
    np.testing.assert_allclose(samples.sum(axis=1), 0.0, atol=1e-12)
