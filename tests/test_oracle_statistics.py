"""Statistical and hydrodynamic pins of the oracle against closed forms.

* LB equipartition (Sec. III, Sec. IV; fluctuating LB thermalises every mode):
  <|j(k)|^2>/N = rho0 kT per Cartesian component and <|rho(k)|^2>/N = rho0 kT / c_s^2
  at every k, except k = 0 (conserved) and the longitudinal momentum at the axis
  Nyquist wave number, which the streaming-collision map leaves invariant.
* SMOL static structure factor, exact for the discrete-time scheme with frozen
  noise: S(q) = 2 kT M (-L_out) |phi(z)|^2 / (1 - |R(z)|^2), z = -lambda, whose
  dt -> 0 limit is the lattice Ornstein-Zernike form kT / (A - K L_SO) of
  Eq. (test2) and the text after it.
* Shear-wave decay rate nu k^2 with nu = c_s^2 (1/omega_s - 1/2) (the viscosity
  of the LB trapezoid scheme, App. B).
"""
import numpy as np
import pytest

import oracle as O

CS2 = 1.0 / 3.0


def _grid(p):
    d = O.d_of(p)
    return (p.nz, p.ny, p.nx) if d == 3 else (p.ny, p.nx)


@pytest.mark.parametrize("lattice,shape,nsteps", [(O.D2Q9, (12, 10, 1), 12000),
                                                  (O.D3Q15, (6, 6, 4), 5000),
                                                  (O.D3Q19, (6, 6, 4), 5000)])
def test_lb_equipartition(lattice, shape, nsteps):
    p = O.make_params(lattice=lattice, coupling=O.LB_ONLY, shape=shape, kT=1e-4, rho0=1.0)
    f, psi = O.init(p)
    c, _ = O.velocities(lattice)
    d = O.d_of(p)
    g = _grid(p)
    O.run(p, f, psi, 0, 200)
    accj = 0.0
    accr = 0.0
    ns = 0
    for n in range(200, nsteps, 2):
        O.run(p, f, psi, n, 2)
        j = (c[:, :d].T.astype(float) @ f).reshape((d,) + g)
        rho = f.sum(axis=0).reshape(g)
        accj = accj + np.abs(np.fft.fftn(j, axes=tuple(range(1, d + 1)))) ** 2
        accr = accr + np.abs(np.fft.fftn(rho)) ** 2
        ns += 1
    N = O.nsites(p)
    Sj = accj / ns / N / (p.rho0 * p.kT)
    Sr = accr / ns / N / (p.rho0 * p.kT / CS2)
    for a in range(d):
        mask = np.ones(g, dtype=bool)
        mask[(0,) * d] = False
        for idx in _staggered_invariants(lattice, g, a):
            assert Sj[a][idx] < 1e-20  # staggered invariant, never excited
            mask[idx] = False
        vals = Sj[a][mask]
        assert abs(vals.mean() - 1) < 0.03
        assert np.all(np.abs(vals - 1) < 0.3)
    mask = np.ones(g, dtype=bool)
    mask[(0,) * d] = False
    assert abs(Sr[mask].mean() - 1) < 0.03


def _staggered_invariants(lattice, g, a):
    """Wave vectors (array indices, axes (z,) y, x) at which momentum component
    a is invariant under the LB (R19): the longitudinal Nyquist mode of every
    lattice, and on D3Q15, whose moving velocities all change the parity of
    x + y + z, also k_a = 0 with the other two components at pi, and
    (pi, pi, pi)."""
    d = len(g)
    half = [L // 2 if L % 2 == 0 else None for L in g]  # Nyquist index per array axis
    ax = d - 1 - a  # array axis of component a
    out = []
    if half[ax] is not None:
        idx = [0] * d
        idx[ax] = half[ax]
        out.append(tuple(idx))
    if lattice == O.D3Q15 and all(h is not None for h in half):
        others = [x for x in range(d) if x != ax]
        idx = [0] * d
        for x in others:
            idx[x] = half[x]
        out.append(tuple(idx))
        out.append(tuple(half))
    return out


def _so_symbol(q, lattice):
    c = np.cos(q)
    if lattice != O.D2Q9:
        return (12 * c.sum(0) + 12 * (c[0] * c[1] + c[0] * c[2] + c[1] * c[2])
                + 8 * c[0] * c[1] * c[2] - 80) / 22
    return c[0] + c[1] + c[0] * c[1] - 3


def _fv_lap(q, lattice):
    s, c = np.sin(q), np.cos(q)
    if lattice == O.D3Q19:
        return -(s[0] ** 2 * (1 + c[1] + c[2]) ** 2 + s[1] ** 2 * (1 + c[0] + c[2]) ** 2
                 + s[2] ** 2 * (1 + c[0] + c[1]) ** 2) / 9
    if lattice == O.D3Q15:
        return -(s[0] ** 2 * (2 + c[1] * c[2]) ** 2 + s[1] ** 2 * (2 + c[0] * c[2]) ** 2
                 + s[2] ** 2 * (2 + c[0] * c[1]) ** 2) / 9
    return -(s[0] ** 2 * (2 + c[1]) ** 2 + s[1] ** 2 * (2 + c[0]) ** 2) / 9


@pytest.mark.parametrize("lattice,smol,shape,nsteps", [(O.D2Q9, O.FD, (16, 12, 1), 16000),
                                                       (O.D2Q9, O.FV, (16, 12, 1), 16000),
                                                       (O.D3Q19, O.FV, (6, 6, 6), 6000)])
def test_smol_static_structure_factor(lattice, smol, shape, nsteps):
    p = O.make_params(lattice=lattice, smol=smol, coupling=O.SMOL_ONLY, shape=shape,
                      kT=1e-3, a=0.5, b=0.0, kappa=0.1, M=0.2)
    f, psi = O.init(p, 0, 0.0)
    d = O.d_of(p)
    g = _grid(p)
    O.run(p, f, psi, 0, 300)
    acc = 0.0
    ns = 0
    for n in range(300, nsteps, 3):
        O.run(p, f, psi, n, 3)
        acc = acc + np.abs(np.fft.fftn(psi.reshape(g))) ** 2
        ns += 1
    S = acc / ns / O.nsites(p)
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(L) * 1.0 for L in g], indexing="ij")
    q = np.array(ks[::-1])  # q[0] is q_x
    lso = _so_symbol(q, lattice)
    lout = lso if smol == O.FD else _fv_lap(q, lattice)
    z = -p.M * (-lout) * (p.a - p.kappa * lso)
    R = 1 + z + z * z / 2
    phi = 1 + z / 2
    with np.errstate(divide="ignore", invalid="ignore"):
        theory = 2 * p.kT * p.M * (-lout) * phi ** 2 / (1 - R ** 2)
    live = np.abs(lout) > 1e-12  # k = 0 and, for FV, the frozen q in {0, pi}^d
    ratio = S[live] / theory[live]
    assert abs(ratio.mean() - 1) < 0.02
    assert np.all(np.abs(ratio - 1) < 0.25)
    # The continuum-time limit is the lattice Ornstein-Zernike law kT/(A - K L):
    oz = p.kT / (p.a - p.kappa * lso)
    assert np.all(np.abs(theory[live] / oz[live] - 1) < 0.25)


@pytest.mark.parametrize("lattice,shape", [(O.D2Q9, (96, 2, 1)), (O.D3Q15, (64, 2, 2)),
                                           (O.D3Q19, (64, 2, 2))])
def test_shear_wave_decay(lattice, shape):
    eta = 0.1
    p = O.make_params(lattice=lattice, coupling=O.LB_ONLY, shape=shape, kT=0.0, eta=eta)
    c, w = O.velocities(lattice)
    d = O.d_of(p)
    N = O.nsites(p)
    x = np.arange(N) % p.nx
    k = 2 * np.pi / p.nx
    U = 1e-4
    u = np.zeros((d, N))
    u[1] = U * np.sin(k * x)
    cu = c[:, :d].astype(float) @ u
    f = w[:, None] * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - (u ** 2).sum(0) / (2 * CS2))
    f = np.ascontiguousarray(f)
    psi = np.zeros(N)

    def amp():
        jy = c[:, 1].astype(float) @ f
        return 2 * (jy * np.sin(k * x)).sum() / N

    O.run(p, f, psi, 0, 100)
    a0 = amp()
    O.run(p, f, psi, 100, 800)
    a1 = amp()
    rate = -np.log(a1 / a0) / 800
    nu = CS2 * (1 / (1 / (0.5 + eta / CS2)) - 0.5)
    assert abs(rate / (nu * k * k) - 1) < 0.01
