"""Pins of the coupled oracle step: conservation laws and the force sign.

* Mass and total psi are conserved to rounding (Sec. I, Sec. V: both
  discretisations are conservative).
* Momentum balance: sum fbar c changes each step by exactly sum F, with F the
  force density (App. B moment relations, force-density reading).  With B = 0
  the central and Gamma gradients make sum F vanish, so momentum is conserved.
* Force sign (reading F = -psi grad mu): with M = 0 and kT = 0 the order
  parameter moves only by advection, the force and the advection exchange
  energy, and viscosity dissipates it, so free energy plus kinetic energy must
  fall at every step.  The opposite sign feeds energy in and blows up.
"""
import numpy as np
import pytest

import oracle as O

CASES = [(O.D2Q9, O.FD, (20, 14, 1)), (O.D2Q9, O.FV, (20, 14, 1)),
         (O.D3Q15, O.FD, (8, 7, 6)), (O.D3Q15, O.FV, (8, 7, 6)),
         (O.D3Q19, O.FD, (8, 7, 6)), (O.D3Q19, O.FV, (8, 7, 6))]


def _momentum(p, f):
    c, _ = O.velocities(p.lattice)
    return (c[:, :O.d_of(p)].T.astype(float) @ f)


@pytest.mark.parametrize("lattice,smol,shape", CASES)
def test_mass_psi_momentum_balance(lattice, smol, shape):
    p = O.make_params(lattice=lattice, smol=smol, shape=shape, a=-0.04, b=0.04, kappa=0.05,
                      kT=1e-4, M=0.1)
    f, psi = O.init(p, 0, 0.3)
    for n in range(12):
        t0 = O.totals(p, f, psi)
        F = O.force(p, psi)
        P0 = _momentum(p, f).sum(axis=1)
        O.step(p, f, psi, n)
        t1 = O.totals(p, f, psi)
        P1 = _momentum(p, f).sum(axis=1)
        assert abs(t1[0] - t0[0]) <= 1e-13 * t0[5]
        assert abs(t1[4] - t0[4]) <= 1e-13 * t0[9]
        scale = np.abs(_momentum(p, f)).sum() + np.abs(F).sum()
        np.testing.assert_allclose(P1 - P0, F.sum(axis=1), atol=1e-13 * scale)


@pytest.mark.parametrize("lattice,smol,shape", CASES)
def test_momentum_conserved_without_quartic_term(lattice, smol, shape):
    p = O.make_params(lattice=lattice, smol=smol, shape=shape, a=0.04, b=0.0, kappa=0.05,
                      kT=1e-4, M=0.1)
    f, psi = O.init(p, 0, 0.3)
    for n in range(8):
        F = O.force(p, psi)
        assert np.abs(F.sum(axis=1)).max() <= 1e-15 * max(1.0, np.abs(F).sum())
        P0 = _momentum(p, f).sum(axis=1)
        O.step(p, f, psi, n)
        P1 = _momentum(p, f).sum(axis=1)
        np.testing.assert_allclose(P1, P0, atol=1e-14 * np.abs(_momentum(p, f)).sum())


@pytest.mark.parametrize("lattice,smol,shape", CASES)
def test_stress_force_conserves_momentum_with_quartic_term(lattice, smol, shape):
    """The divergence of the stress of Eq. (muf) sums to zero over the lattice
    for any B (every term is a difference of shifted copies), where -psi grad
    mu does not; the momentum of a two-phase run is then constant."""
    kw = dict(lattice=lattice, smol=smol, shape=shape, a=-0.04, b=0.04, kappa=0.05, kT=1e-4,
              M=0.1)
    p = O.make_params(force_form=O.FORCE_STRESS, **kw)
    pg = O.make_params(**kw)
    f, psi = O.init(p, 0, 0.3)
    F, Fg = O.force(p, psi), O.force(pg, psi)
    assert np.abs(F.sum(axis=1)).max() <= 1e-15 * np.abs(F).sum()
    assert np.abs(Fg.sum(axis=1)).max() > 1e-9 * np.abs(Fg).sum()
    sig = O.stress(p, psi)
    np.testing.assert_allclose(sig, sig.transpose(1, 0, 2), rtol=1e-15, atol=1e-18)
    for n in range(8):
        P0 = _momentum(p, f).sum(axis=1)
        O.step(p, f, psi, n)
        P1 = _momentum(p, f).sum(axis=1)
        np.testing.assert_allclose(P1, P0, atol=1e-14 * np.abs(_momentum(p, f)).sum())


@pytest.mark.parametrize("lattice,smol", [(O.D2Q9, O.FD), (O.D2Q9, O.FV), (O.D3Q19, O.FD),
                                          (O.D3Q19, O.FV), (O.D3Q15, O.FV)])
def test_stress_force_is_psi_grad_mu_in_the_continuum(lattice, smol):
    """On a smooth field the two discrete forces differ by O(h^2): doubling
    the resolution of the same profile cuts their difference about 4x
    (Eq. muf: div sigma = psi grad mu in the continuum)."""
    errs = []
    for L in (24, 48):
        d = 2 if lattice == O.D2Q9 else 3
        shape = (L, L, 1) if d == 2 else (L, L, 8)
        kw = dict(lattice=lattice, smol=smol, shape=shape, a=-0.3, b=0.5, kappa=0.8)
        p, pg = O.make_params(force_form=O.FORCE_STRESS, **kw), O.make_params(**kw)
        N = O.nsites(p)
        x = np.arange(N) % L
        y = (np.arange(N) // L) % L
        h = 2 * np.pi / L
        psi = 0.6 * np.sin(h * x) + 0.4 * np.cos(h * y) * np.sin(h * x + 0.3)
        # the same physical field at twice the resolution: gradients scale by h
        F, Fg = O.force(p, psi), O.force(pg, psi)
        errs.append(np.abs(F - Fg).max() / np.abs(Fg).max())
    ratio = errs[0] / errs[1]
    assert errs[0] < 0.08
    assert 3.2 < ratio < 4.8, (errs, ratio)


def _energy(p, f, psi):
    F = O.force(p, psi)
    rho = f.sum(axis=0)
    mom = _momentum(p, f) + F / 2
    ke = 0.5 * (mom ** 2).sum(axis=0) / rho
    fe = p.a * psi ** 2 / 2 + p.b * psi ** 4 / 4 - 0.5 * p.kappa * psi * O.laplacian(p, psi)
    return fe.sum() + ke.sum()


@pytest.mark.parametrize("lattice,smol,shape", [(O.D2Q9, O.FD, (24, 24, 1)),
                                                (O.D2Q9, O.FV, (24, 24, 1)),
                                                (O.D3Q19, O.FD, (10, 10, 10)),
                                                (O.D3Q19, O.FV, (10, 10, 10)),
                                                (O.D3Q15, O.FV, (10, 10, 10))])
def test_force_sign_dissipates_energy(lattice, smol, shape):
    p = O.make_params(lattice=lattice, smol=smol, shape=shape, a=-0.04, b=0.04, kappa=0.05,
                      kT=0.0, M=0.0)
    f, psi = O.init(p, 0, 0.5)
    E = [_energy(p, f, psi)]
    for n in range(150):
        O.step(p, f, psi, n)
        E.append(_energy(p, f, psi))
    E = np.array(E)
    assert np.all(np.diff(E) < 0)
    assert E[-1] < 0.7 * E[0]


def test_two_phase_run_stays_bounded():
    """Two flat interfaces with the paper's capillary parameters (Sec. VI.C:
    -A = B = 0.05, K = 0.2, M = 0.1, tau = 0.45 i.e. eta = 0.15): the Runge-Kutta
    stages see the velocity of their own time level, so the staggered
    longitudinal LB mode cannot pump the interfaces and the flow stays at the
    level of the interface's spurious currents.  (With u^n frozen over both
    stages this run diverges near step 1200.)"""
    for smol in (O.FV, O.FD):
        p = O.make_params(lattice=O.D2Q9, smol=smol, shape=(48, 48, 1), a=-0.05, b=0.05,
                          kappa=0.2, M=0.1, kT=1e-5, eta=0.15)
        f, psi = O.init(p, 1, 1e-3)
        umax = []
        for k in range(8):
            O.run(p, f, psi, k * 250, 250)
            umax.append(np.abs(O.velocity(p, f, O.force(p, psi))).max())
        assert np.all(np.isfinite(umax)) and max(umax) < 0.05
        assert np.abs(psi).max() < 1.1
