"""Pins of the oracle with solid walls across the last axis (the closing
remark of Sec. V.B: the finite-volume SMOL admits walls and shear
boundaries).  Reading: every stencil link that crosses a wall is removed (no
flux through it), and the LB populations that would leave through a wall
return to their site reversed (halfway bounce-back, with Ladd's term for a
moving wall).

* The discrete operators with walls, as matrices built column by column from
  unit fields: Div = -Grad^T (so the diffusion operator Div Grad and the
  noise covariance 2 kT M Div Div^T = -2 kT M Div Grad keep the
  fluctuation-dissipation balance of the periodic scheme), the
  Shinozaki-Oono Laplacian symmetric with zero row sums, Grad of a constant
  zero, and all equal to the periodic operators away from the walls.
* Couette flow: the fluid between walls moving at -U and +U relaxes to the
  exact linear profile u_x = -U + 2U (h + 1/2)/L, the walls half a spacing
  beyond the end layers.
* Mass and psi are conserved to rounding with walls, noise and two phases;
  with M = 0 and kT = 0 free plus kinetic energy falls at every step between
  static walls.
"""
import numpy as np
import pytest

import oracle as O

CASES = [(O.D2Q9, (6, 7, 1)), (O.D3Q19, (4, 5, 6)), (O.D3Q15, (4, 5, 6))]


def _matrices(p):
    N = O.nsites(p)
    d = O.d_of(p)
    G = np.zeros((d * N, N))
    L = np.zeros((N, N))
    Dv = np.zeros((N, d * N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        G[:, k] = O.gradient(p, e).reshape(-1)
        L[:, k] = O.laplacian(p, e)
    for k in range(d * N):
        e = np.zeros((d, N))
        e.reshape(-1)[k] = 1.0
        Dv[:, k] = O.divergence(p, e)
    return G, L, Dv


@pytest.mark.parametrize("lattice,shape", CASES)
def test_wall_operators_are_adjoint_and_local(lattice, shape):
    p = O.make_params(lattice=lattice, smol=O.FV, shape=shape, walls=1)
    pp = O.make_params(lattice=lattice, smol=O.FV, shape=shape)
    G, L, Dv = _matrices(p)
    Gp, Lp, Dvp = _matrices(pp)
    np.testing.assert_allclose(Dv, -G.T, rtol=0, atol=1e-15)
    np.testing.assert_allclose(L, L.T, rtol=0, atol=1e-15)
    np.testing.assert_allclose(L.sum(axis=1), 0.0, atol=1e-14)
    N = O.nsites(p)
    np.testing.assert_allclose(G @ np.ones(N), 0.0, atol=1e-15)
    # the FV diffusion operator is symmetric negative semi-definite
    K = Dv @ G
    np.testing.assert_allclose(K, K.T, atol=1e-14)
    assert np.linalg.eigvalsh(K).max() < 1e-13
    # rows of sites two or more layers from the walls are the periodic ones
    d = O.d_of(p)
    h = (np.arange(N) // (shape[0] * shape[1])) if d == 3 else (np.arange(N) // shape[0])
    Lh = shape[2] if d == 3 else shape[1]
    inner = (h >= 2) & (h < Lh - 2)
    np.testing.assert_allclose(L[inner], Lp[inner], atol=1e-15)
    np.testing.assert_allclose(Dv[inner], Dvp[inner], atol=1e-15)
    for a in range(d):
        np.testing.assert_allclose(G[a * N:(a + 1) * N][inner], Gp[a * N:(a + 1) * N][inner],
                                   atol=1e-15)
    # and the walls do change the rows at the end layers
    assert np.abs(L[h == 0] - Lp[h == 0]).max() > 0.01


@pytest.mark.parametrize("lattice,shape", CASES)
def test_wall_noise_is_the_divergence_of_node_noise(lattice, shape):
    """N = Div xi with the wall divergence: its covariance is
    2 kT M Div Div^T = -2 kT M Div Grad, and it sums to zero."""
    p = O.make_params(lattice=lattice, smol=O.FV, shape=shape, walls=1, kT=1e-4, M=0.2)
    _, _, Dv = _matrices(p)
    N = O.nsites(p)
    d = O.d_of(p)
    amp = np.sqrt(2 * p.kT * p.M)
    xi = np.array([[amp * O.normal(p.seed, s, 7, O.TAG_SMOL, a) for s in range(N)]
                   for a in range(d)])
    noise = O.smol_noise(p, 7)
    np.testing.assert_allclose(noise, Dv @ xi.reshape(-1), rtol=0, atol=1e-16)
    assert abs(noise.sum()) < 1e-16 * N


@pytest.mark.parametrize("lattice,shape", [(O.D2Q9, (4, 10, 1)), (O.D3Q19, (4, 4, 10)),
                                           (O.D3Q15, (4, 4, 10))])
def test_couette_profile(lattice, shape):
    """With every mode relaxed at the shear rate the linear profile is exact
    to rounding; with other bulk and ghost rates the O(U^2) terms of the
    equilibrium add a density adjustment of relative size ~ U^2 (not
    tested here)."""
    U = 0.02
    ws = 1 / (0.5 + 3 * 0.1)
    p = O.make_params(lattice=lattice, smol=O.FV, coupling=O.LB_ONLY, shape=shape, kT=0.0,
                      eta=0.1, walls=1, u_wall=(-U, 0, 0, U, 0, 0), omega_bulk=ws,
                      omega_ghost=ws)
    f, psi = O.init(p, 0, 0.0)
    O.run(p, f, psi, 0, 6000)
    u = O.velocity(p, f, np.zeros((O.d_of(p), O.nsites(p))))
    d = O.d_of(p)
    L = shape[2] if d == 3 else shape[1]
    h = (np.arange(O.nsites(p)) // (shape[0] * shape[1])) if d == 3 \
        else (np.arange(O.nsites(p)) // shape[0])
    want = -U + 2 * U * (h + 0.5) / L
    np.testing.assert_allclose(u[0], want, rtol=0, atol=1e-10)
    np.testing.assert_allclose(u[1:], 0.0, atol=1e-12)


@pytest.mark.parametrize("lattice,shape", [(O.D2Q9, (12, 10, 1)), (O.D3Q19, (6, 5, 8)),
                                           (O.D3Q15, (6, 5, 8))])
def test_wall_conservation(lattice, shape):
    p = O.make_params(lattice=lattice, smol=O.FV, shape=shape, a=-0.04, b=0.04, kappa=0.05,
                      kT=1e-4, M=0.1, walls=1, u_wall=(0.01, 0.0, 0.0, -0.01, 0.0, 0.0))
    f, psi = O.init(p, 1, 0.05)
    t0 = O.totals(p, f, psi)
    O.run(p, f, psi, 0, 40)
    t1 = O.totals(p, f, psi)
    assert abs(t1[0] - t0[0]) <= 1e-13 * t0[5]
    assert abs(t1[4] - t0[4]) <= 1e-13 * t0[9]


def _energy(p, f, psi):
    c, _ = O.velocities(p.lattice)
    F = O.force(p, psi)
    rho = f.sum(axis=0)
    mom = c[:, :O.d_of(p)].T.astype(float) @ f + F / 2
    ke = 0.5 * (mom ** 2).sum(axis=0) / rho
    fe = p.a * psi ** 2 / 2 + p.b * psi ** 4 / 4 - 0.5 * p.kappa * psi * O.laplacian(p, psi)
    return fe.sum() + ke.sum()


@pytest.mark.parametrize("lattice,shape", [(O.D2Q9, (20, 16, 1)), (O.D3Q19, (8, 8, 10))])
def test_wall_energy_dissipation(lattice, shape):
    p = O.make_params(lattice=lattice, smol=O.FV, shape=shape, a=-0.04, b=0.04, kappa=0.05,
                      kT=0.0, M=0.0, walls=1)
    f, psi = O.init(p, 0, 0.5)
    E = [_energy(p, f, psi)]
    for n in range(120):
        O.step(p, f, psi, n)
        E.append(_energy(p, f, psi))
    E = np.array(E)
    assert np.all(np.diff(E) < 0)
    assert E[-1] < 0.7 * E[0]


@pytest.mark.parametrize("lattice,shape", [(O.D2Q9, (9, 11, 1)), (O.D3Q19, (5, 5, 7)),
                                           (O.D3Q15, (5, 5, 7))])
def test_wall_noise_keeps_the_boltzmann_distribution(lattice, shape):
    """Fluctuation-dissipation balance with walls: the stationary covariance
    of the oracle's SMOL between walls (B = 0, no flow, Heun with frozen
    noise) tends to the Boltzmann covariance kT H^-1 of the discrete free
    energy, H = A - K L_SO (on the fluctuations of zero total), as the time
    step shrinks (M -> 0 at fixed A, K), with the O(M^2) error of the
    discrete-time scheme.  A wall rule that broke Div = -Grad^T or the
    symmetry of L_SO would leave an O(1) deviation."""
    from tests import theory as T
    devs = []
    for M in (0.1, 0.01):
        p = O.make_params(lattice=lattice, smol=O.FV, coupling=O.SMOL_ONLY, shape=shape, a=0.04,
                          b=0.0, kappa=0.05, M=M, kT=1e-5, walls=1)
        L, H, Dv = T.smol_linear_operators(p)
        C = T.stationary_covariance(L, H, Dv, 1e-5, M)
        N = O.nsites(p)
        P = np.eye(N) - np.ones((N, N)) / N
        Cb = 1e-5 * P @ np.linalg.pinv(P @ H @ P, rcond=1e-10, hermitian=True) @ P
        devs.append(np.abs(C - Cb).max() / np.abs(Cb).max())
    assert devs[0] < 1e-3 and devs[1] < 1e-5
    assert 50 < devs[0] / devs[1] < 200  # second order in the step
    # the walls shape the profile: the end layers fluctuate more than the bulk
    d = O.d_of(p)
    per = np.diag(C).reshape(shape[d - 1], -1).mean(axis=1)
    assert per[0] > 1.2 * per[len(per) // 2] and abs(per[0] - per[-1]) < 1e-12 * per[0]


@pytest.mark.parametrize("lattice,shape", [(O.D2Q9, (9, 11, 1)), (O.D3Q19, (5, 5, 7))])
def test_stationary_covariance_matches_the_discrete_closed_form(lattice, shape):
    """The covariance machinery on a periodic lattice at a finite step
    (M = 0.1) against the exact discrete-time static structure factor
    2 kT M (-L_out) |Phi(z)|^2 / (1 - |R(z)|^2) of each Fourier mode (odd
    sides: only q = 0 is conserved)."""
    from tests import theory as T
    p = O.make_params(lattice=lattice, smol=O.FV, coupling=O.SMOL_ONLY, shape=shape, a=0.04,
                      b=0.0, kappa=0.05, M=0.1, kT=1e-5)
    L, H, Dv = T.smol_linear_operators(p)
    C = T.stationary_covariance(L, H, Dv, 1e-5, 0.1)
    nx, ny, nz = shape
    d = O.d_of(p)
    idx = np.arange(O.nsites(p))
    xyz = [idx % nx, (idx // nx) % ny, idx // (nx * ny)]
    for m in [(1, 0, 0), (0, 2, 0), (1, 1, 0), (2, 3, 0)] + ([(1, 0, 2), (2, 1, 3)] if d == 3 else []):
        q = np.array([2 * np.pi * m[k] / shape[k] for k in range(3)])[:d]
        v = np.exp(1j * sum(q[k] * xyz[k] for k in range(d)))
        got = np.real(np.conj(v) @ C @ v) / O.nsites(p)
        want = T.smol_static_sk(q.reshape(d, 1), lattice, O.FV, 0.1, 0.04, 0.05, 1e-5)[0]
        assert abs(got / want - 1) < 1e-10, (m, got, want)
