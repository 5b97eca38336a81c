"""Pins of the full-coupling Runge-Kutta stages of the oracle (Sec. V: the
SMOL noise is held constant through the step; by the stage-velocity reading,
each stage advects with the velocity of its own time level: u^n at t_n, the
velocity of the streamed populations at t_{n+1}, and their mean at the RK4
midpoints).

On fields that vary along x only, every stencil of the method reduces to a
one-dimensional operator with a closed form: the Shinozaki-Oono Laplacian to
the three-point Laplacian l = phi(x+1) - 2 phi(x) + phi(x-1) (its symbol with
the transverse cosines set to 1 is 2(cos q - 1)), both the central and the FV
gradient Gamma = (1/c_s^2) sum_i w_i c_i to the central difference
d = (phi(x+1) - phi(x-1))/2, and the FV Laplacian Gamma.Gamma to d d.  With
B = 0 and kT = 0 the SMOL right-hand side is linear in phi,
    G(phi; u) = -d(u phi) + M L_out (A phi - K l phi),   L_out = l (FD), d d (FV),
and one step is the Runge-Kutta combination of these n x n matrices with the
stage velocities.  The tests build the matrices from these one-dimensional
forms, take the classical Butcher tableaux of Euler, Heun and RK4, and compare
the oracle's psi^{n+1} with the result, so that a wrong stage velocity,
weight or time level in the oracle's coupled step shows up far above
rounding.  The velocities come from the oracle's LB (pinned elsewhere) before
and after its step.

The physical pins of the same stages: with M = 0 and kT = 0 the reversible
coupling only exchanges energy and viscosity dissipates it, so free plus
kinetic energy falls at every step for RK4 as for Heun; and a two-phase run
with RK4 stays bounded.
"""
import numpy as np
import pytest

import oracle as O

# Butcher tableaux: stage velocity label, stage offsets, weights.
TABLEAU = {
    1: (["n"], [], [1.0]),
    2: (["n", "n1"], [1.0], [0.5, 0.5]),
    4: (["n", "h", "h", "n1"], [0.5, 0.5, 1.0], [1 / 6, 1 / 3, 1 / 3, 1 / 6]),
}


def _circ(n, taps):
    m = np.zeros((n, n))
    for off, v in taps.items():
        for x in range(n):
            m[x, (x + off) % n] += v
    return m


def _rk_step(G, psi, rk, un, u1):
    labels, a, b = TABLEAU[rk]
    vel = {"n": un, "n1": u1, "h": 0.5 * (un + u1)}
    ks = []
    for j, lab in enumerate(labels):
        phi = psi if j == 0 else psi + a[j - 1] * ks[-1]
        ks.append(G(phi, vel[lab]))
    return psi + sum(bj * kj for bj, kj in zip(b, ks))


@pytest.mark.parametrize("lattice,shape", [(O.D2Q9, (24, 4, 1)), (O.D3Q19, (20, 4, 4)),
                                           (O.D3Q15, (20, 4, 4))])
@pytest.mark.parametrize("smol", [O.FD, O.FV])
@pytest.mark.parametrize("rk", [1, 2, 4])
def test_full_coupling_stages_on_one_dimensional_fields(lattice, shape, smol, rk):
    nx = shape[0]
    A, K, M = 0.04, 0.05, 0.1
    p = O.make_params(lattice=lattice, smol=smol, rk_stages=rk, shape=shape, a=A, b=0.0,
                      kappa=K, M=M, kT=0.0, eta=0.1)
    N = O.nsites(p)
    D = O.d_of(p)
    c, w = O.velocities(lattice)
    x = np.arange(N) % nx
    # populations at equilibrium with a longitudinal flow u_x(x); psi(x) smooth
    ux = 0.02 * np.sin(2 * np.pi * x / nx) + 0.01 * np.cos(4 * np.pi * x / nx + 0.4)
    f = np.zeros((len(w), N))
    for i in range(len(w)):
        cu = c[i, 0] * ux
        f[i] = w[i] * (1 + 3 * cu + 4.5 * cu * cu - 1.5 * ux * ux)
    amp = np.random.default_rng(5).standard_normal(6)
    xs = np.arange(nx)
    psi1 = 0.3 * sum(amp[k] * np.cos(2 * np.pi * (k + 1) * xs / nx + k) for k in range(6))
    psi = np.ascontiguousarray(psi1[x])

    d = _circ(nx, {1: 0.5, -1: -0.5})
    lap = _circ(nx, {1: 1.0, 0: -2.0, -1: 1.0})
    lout = lap if smol == O.FD else d @ d

    def G(phi, u):
        return -d @ (u * phi) + M * (lout @ (A * phi - K * (lap @ phi)))

    for n in range(6):
        F = O.force(p, psi)
        un = O.velocity(p, f, F)
        prev = psi[:nx].copy()
        O.step(p, f, psi, n)
        u1 = O.velocity(p, f, F)  # streamed populations with the time-n force
        # the fields stay functions of x alone, with no transverse flow
        assert np.abs(un[1:D]).max() < 1e-15 and np.abs(u1[1:D]).max() < 1e-15
        rows = psi.reshape(-1, nx)
        assert np.abs(rows - rows[0]).max() < 1e-15
        assert np.abs(un[0] - un[0, :nx][x]).max() < 1e-15
        want = _rk_step(G, prev, rk, un[0, :nx], u1[0, :nx])
        err = np.abs(rows[0] - want).max() / np.abs(want).max()
        assert err <= 1e-13, (n, err)
        # the velocities of the two time levels differ: the stage velocity matters
        assert np.abs(u1[0, :nx] - un[0, :nx]).max() > 1e-5


def test_wrong_stage_velocity_would_be_seen():
    """The one-dimensional check separates the readings: evaluating RK4's
    mid stages with u^n, or every stage with u^n, moves psi^{n+1} by far more
    than the bar above."""
    nx = 24
    A, K, M = 0.04, 0.05, 0.1
    d = _circ(nx, {1: 0.5, -1: -0.5})
    lap = _circ(nx, {1: 1.0, 0: -2.0, -1: 1.0})

    def G(phi, u):
        return -d @ (u * phi) + M * (lap @ (A * phi - K * (lap @ phi)))

    xs = np.arange(nx)
    psi = np.cos(2 * np.pi * xs / nx) + 0.5 * np.sin(6 * np.pi * xs / nx)
    un = 0.02 * np.sin(2 * np.pi * xs / nx)
    u1 = 0.9 * un
    good = _rk_step(G, psi, 4, un, u1)
    frozen = _rk_step(G, psi, 4, un, un)
    assert np.abs(good - frozen).max() / np.abs(good).max() > 1e-6


def _momentum(p, f):
    c, _ = O.velocities(p.lattice)
    return c[:, :O.d_of(p)].T.astype(float) @ f


def _energy(p, f, psi):
    F = O.force(p, psi)
    rho = f.sum(axis=0)
    mom = _momentum(p, f) + F / 2
    ke = 0.5 * (mom ** 2).sum(axis=0) / rho
    fe = p.a * psi ** 2 / 2 + p.b * psi ** 4 / 4 - 0.5 * p.kappa * psi * O.laplacian(p, psi)
    return fe.sum() + ke.sum()


@pytest.mark.parametrize("lattice,smol,shape", [(O.D2Q9, O.FD, (24, 24, 1)),
                                                (O.D2Q9, O.FV, (24, 24, 1)),
                                                (O.D3Q19, O.FV, (10, 10, 10))])
def test_rk4_full_coupling_dissipates_energy(lattice, smol, shape):
    p = O.make_params(lattice=lattice, smol=smol, shape=shape, a=-0.04, b=0.04, kappa=0.05,
                      kT=0.0, M=0.0, rk_stages=4)
    f, psi = O.init(p, 0, 0.5)
    E = [_energy(p, f, psi)]
    for n in range(150):
        O.step(p, f, psi, n)
        E.append(_energy(p, f, psi))
    E = np.array(E)
    assert np.all(np.diff(E) < 0)
    assert E[-1] < 0.7 * E[0]


def test_rk4_two_phase_run_stays_bounded():
    """The capillary parameters of Sec. VI.C (-A = B = 0.05, K = 0.2, M = 0.1,
    eta = 0.15) with RK4 stages: the flow stays at the level of the
    interfaces' spurious currents over 2000 steps."""
    for smol in (O.FV, O.FD):
        p = O.make_params(lattice=O.D2Q9, smol=smol, shape=(48, 48, 1), a=-0.05, b=0.05,
                          kappa=0.2, M=0.1, kT=1e-5, eta=0.15, rk_stages=4)
        f, psi = O.init(p, 1, 1e-3)
        umax = []
        for k in range(8):
            O.run(p, f, psi, k * 250, 250)
            umax.append(np.abs(O.velocity(p, f, O.force(p, psi))).max())
        assert np.all(np.isfinite(umax)) and max(umax) < 0.05
        assert np.abs(psi).max() < 1.1
