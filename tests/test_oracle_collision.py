"""Pins of the oracle's FLBE collision (App. B) on single sites.

The oracle collides in a w-orthonormal mode basis (Gram-Schmidt over
monomials) with separate bulk, shear and ghost rates and noise on every
non-conserved mode.  These tests pin it against formulas written in
population space, independent of the mode basis:
  * all rates equal, kT = 0: the paper's single-relaxation update below
    Eq. (barlin), fbar* = fbar + dt/(tau + dt/2) [-(fbar - f0) + tau Phi];
  * ghosts projected out, kT = 0: the paper's Eq. (bab);
  * unequal rates: moment-by-moment relaxation of the trace and traceless
    stress and of the ghost subspace;
  * noise enters only the non-conserved moments, with variance rho0 kT (1 - gamma^2)/c_s^2
    per orthonormal mode.
"""
import numpy as np
import pytest

import oracle as O

CS2 = 1.0 / 3.0


def _lat(lattice):
    c, w = O.velocities(lattice)
    d = 2 if lattice == O.D2Q9 else 3
    return c[:, :d].astype(float), w, d


def _rand_site(lattice, rng):
    c, w, d = _lat(lattice)
    fbar = w * (1.0 + 0.2 * rng.standard_normal(len(w)))
    F = 0.01 * rng.standard_normal(d)
    return fbar, F


def _equilibrium(c, w, rho, u):
    cu = c @ u
    return w * rho * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - (u @ u) / (2 * CS2))


def _Q(c):
    d = c.shape[1]
    return np.einsum("ia,ib->iab", c, c) - CS2 * np.eye(d)[None]


def _forcing(c, w, u, F):
    # Phi_i = w_i [c.F / c_s^2 + (uF + Fu):Q_i / (2 c_s^4)]
    Q = _Q(c)
    T = np.outer(u, F) + np.outer(F, u)
    return w * (c @ F / CS2 + np.einsum("iab,ab->i", Q, T) / (2 * CS2 ** 2))


def _eta_for(omega, rho0=1.0):
    return (1.0 / omega - 0.5) * rho0 * CS2


@pytest.mark.parametrize("lattice", [O.D2Q9, O.D3Q15, O.D3Q19])
def test_basis_structure(lattice):
    E = O.basis(lattice)
    c, w, d = _lat(lattice)
    q = len(w)
    np.testing.assert_allclose((E * w) @ E.T, np.eye(q), atol=1e-14)
    np.testing.assert_allclose(E[0], 1.0, atol=1e-15)
    for a in range(d):
        np.testing.assert_allclose(E[1 + a], c[:, a] / np.sqrt(CS2), atol=1e-14)
    # Every ghost mode is orthogonal to the second-order equilibrium and to
    # every second moment (Q_ab), i.e. ghosts carry no hydrodynamic content.
    nstress = 3 if d == 2 else 6
    rng = np.random.default_rng(1)
    Q = _Q(c)
    for _ in range(5):
        feq = _equilibrium(c, w, 1 + 0.1 * rng.standard_normal(), 0.1 * rng.standard_normal(d))
        m = E @ feq
        np.testing.assert_allclose(m[1 + d + nstress:], 0.0, atol=1e-15)
    for a in range(d):
        for b in range(d):
            np.testing.assert_allclose((E[1 + d + nstress:] * w) @ Q[:, a, b], 0.0, atol=1e-15)
    # The bulk mode is the trace of Q, the shear modes are traceless.
    trQ = np.einsum("iaa->i", Q)
    bulk = E[1 + d]
    np.testing.assert_allclose(np.abs((bulk * w) @ trQ) / np.sqrt((trQ ** 2 * w).sum()), 1.0,
                               atol=1e-14)
    for k in range(2 + d, 1 + d + nstress):
        assert abs((E[k] * w) @ trQ) < 1e-14


@pytest.mark.parametrize("lattice", [O.D2Q9, O.D3Q15, O.D3Q19])
def test_equal_rates_is_single_relaxation_update(lattice):
    rng = np.random.default_rng(11)
    c, w, d = _lat(lattice)
    for omega in (0.7, 1.0, 1.6):
        p = O.make_params(lattice=lattice, eta=_eta_for(omega), omega_bulk=omega,
                          omega_ghost=omega, kT=0.0)
        for _ in range(10):
            fbar, F = _rand_site(lattice, rng)
            rho = fbar.sum()
            u = (fbar @ c + F / 2) / rho
            tau = 1 / omega - 0.5
            expect = fbar + omega * (-(fbar - _equilibrium(c, w, rho, u))
                                     + tau * _forcing(c, w, u, F))
            got = O.collide(p, fbar, F, np.zeros(16))
            np.testing.assert_allclose(got, expect, atol=2e-15)


@pytest.mark.parametrize("lattice", [O.D2Q9, O.D3Q15, O.D3Q19])
def test_ghost_projection_is_paper_bab(lattice):
    rng = np.random.default_rng(12)
    c, w, d = _lat(lattice)
    Q = _Q(c)
    for omega in (0.8, 1.25, 1.9):
        p = O.make_params(lattice=lattice, eta=_eta_for(omega), omega_bulk=omega,
                          omega_ghost=1.0, kT=0.0)
        tau = 1 / omega - 0.5
        for _ in range(10):
            fbar, F = _rand_site(lattice, rng)
            rho = fbar.sum()
            v = (fbar @ c + F / 2) / rho
            A = fbar @ c + F
            S = np.einsum("i,iab->ab", fbar, Q)
            B = S + omega * (-S + rho * np.outer(v, v) + tau * (np.outer(v, F) + np.outer(F, v)))
            expect = w * (rho + c @ A / CS2 + np.einsum("iab,ab->i", Q, B) / (2 * CS2 ** 2))
            got = O.collide(p, fbar, F, np.zeros(16))
            np.testing.assert_allclose(got, expect, atol=2e-15)


def _moments(c, w, f):
    Q = _Q(c)
    rho = f.sum()
    j = f @ c
    Pi = np.einsum("i,iab->ab", f, Q)
    hydro = w * (rho + c @ j / CS2 + np.einsum("iab,ab->i", Q, Pi) / (2 * CS2 ** 2))
    return rho, j, Pi, f - hydro


@pytest.mark.parametrize("lattice", [O.D2Q9, O.D3Q15, O.D3Q19])
def test_unequal_rates_relax_each_moment(lattice):
    rng = np.random.default_rng(13)
    c, w, d = _lat(lattice)
    ws, wb, wg = 1.25, 0.9, 1.4
    p = O.make_params(lattice=lattice, eta=_eta_for(ws), omega_bulk=wb, omega_ghost=wg, kT=0.0)
    I = np.eye(d)
    for _ in range(10):
        fbar, F = _rand_site(lattice, rng)
        rho, j, Pi, ghost = _moments(c, w, fbar)
        u = (j + F / 2) / rho
        got = O.collide(p, fbar, F, np.zeros(16))
        rho2, j2, Pi2, ghost2 = _moments(c, w, got)
        assert abs(rho2 - rho) < 1e-15
        np.testing.assert_allclose(j2, j + F, atol=1e-15)
        Peq = rho * np.outer(u, u)
        Src = np.outer(u, F) + np.outer(F, u)
        tr = lambda T: np.trace(T) / d * I
        tl = lambda T: T - tr(T)
        gs, gb = 1 - ws, 1 - wb
        expect = (Peq + gs * tl(Pi - Peq) + gb * tr(Pi - Peq)
                  + 0.5 * (1 + gs) * tl(Src) + 0.5 * (1 + gb) * tr(Src))
        np.testing.assert_allclose(Pi2, expect, atol=2e-15)
        np.testing.assert_allclose(ghost2, (1 - wg) * ghost, atol=2e-15)


@pytest.mark.parametrize("lattice", [O.D2Q9, O.D3Q15, O.D3Q19])
def test_noise_only_in_nonconserved_modes(lattice):
    rng = np.random.default_rng(14)
    c, w, d = _lat(lattice)
    q = len(w)
    ws, wb, wg = 1.25, 1.0, 1.0
    rho0, kT = 1.3, 1e-3
    p = O.make_params(lattice=lattice, eta=_eta_for(ws, rho0), omega_bulk=wb, omega_ghost=wg,
                      kT=kT, rho0=rho0)
    p0 = O.make_params(lattice=lattice, eta=_eta_for(ws, rho0), omega_bulk=wb, omega_ghost=wg,
                       kT=0.0, rho0=rho0)
    fbar, F = _rand_site(lattice, rng)
    base = O.collide(p0, fbar, F, np.zeros(16))
    E = O.basis(lattice)
    nr = q - d - 1
    # Unit normal in slot k moves exactly mode k+d+1 by sigma_k.
    for k in range(nr):
        r = np.zeros(16)
        r[k] = 1.0
        delta = O.collide(p, fbar, F, r) - base
        m = E @ delta
        gamma = 1 - (wb if k == 0 else (ws if k < (3 if d == 2 else 6) else wg))
        sigma = np.sqrt((1 - gamma ** 2) * rho0 * kT / CS2)
        expect = np.zeros(q)
        expect[k + d + 1] = sigma
        np.testing.assert_allclose(m, expect, atol=1e-15)
