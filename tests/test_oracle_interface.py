"""The zero-temperature interface (Sec. II.A and Sec. VI.C, Eqs. tanh and
intthick): started from two flat tanh profiles, the coupled oracle must relax
to the lattice's own equilibrium, the profile psi(y) on which the discrete
chemical potential mu = A psi + B psi^3 - K L psi is uniform, at rest.  For a
profile that varies along y only, the 2-D Shinozaki-Oono-type Laplacian
reduces exactly to the 1-D second difference psi(y+1) + psi(y-1) - 2 psi(y),
so the equilibrium is the solution of a 1-D nonlinear system, found here by
Newton's method with the total of psi fixed (independent of the oracle)."""
import numpy as np

import oracle as O


def _newton_profile(psi0, a, b, kappa, tol=1e-14):
    n = psi0.size
    psi = psi0.copy()
    total = psi0.sum()
    lam = 0.0
    for _ in range(100):
        lap = np.roll(psi, 1) + np.roll(psi, -1) - 2 * psi
        r = np.concatenate([a * psi + b * psi ** 3 - kappa * lap - lam, [psi.sum() - total]])
        J = np.zeros((n + 1, n + 1))
        idx = np.arange(n)
        J[idx, idx] = a + 3 * b * psi ** 2 + 2 * kappa
        J[idx, (idx + 1) % n] -= kappa
        J[idx, (idx - 1) % n] -= kappa
        J[idx, n] = -1.0
        J[n, :n] = 1.0
        d = np.linalg.solve(J, -r)
        psi += d[:n]
        lam += d[n]
        if np.abs(d).max() < tol:
            break
    return psi, lam


def test_zero_temperature_interfaces_relax_to_the_discrete_equilibrium():
    """Two interfaces started on lattice sites (y = L/4, 3L/4) sit on a saddle
    of the lattice's pinning potential: rounding breaks the symmetry, both
    translate together (the fluid moves with them; total momentum is not
    conserved when B != 0) and they come to rest half-way between sites.
    The relaxed state must be the discrete equilibrium next to it: uniform mu,
    zero velocity, the Newton profile, bond-centred zero crossings."""
    nx, ny = 4, 32
    a, b, kappa = -0.04, 0.04, 0.05
    p = O.make_params(lattice=O.D2Q9, smol=O.FD, shape=(nx, ny, 1), a=a, b=b, kappa=kappa,
                      M=0.1, kT=0.0, eta=0.1, seed=5)
    f, psi = O.init(p, 1, 0.0)
    col0 = psi.reshape(ny, nx)[:, 0].copy()
    O.run(p, f, psi, 0, 60000)
    g = psi.reshape(ny, nx)
    assert np.abs(g - g[:, :1]).max() < 1e-13  # still x-independent
    prof = g[:, 0]
    assert abs(prof.sum() - col0.sum()) < 1e-11 * np.abs(col0).sum()
    ref, lam = _newton_profile(prof, a, b, kappa)
    mu = O.chemical_potential(p, psi)
    assert np.abs(mu - lam).max() < 1e-9
    assert np.abs(prof - ref).max() < 1e-9
    u = O.velocity(p, f, O.force(p, psi))
    assert np.abs(u).max() < 1e-9
    s_ = np.sign(ref)
    k = np.where(s_[:-1] * s_[1:] <= 0)[0]
    zeros = np.array([kk + ref[kk] / (ref[kk] - ref[kk + 1]) for kk in k])
    assert np.allclose(zeros % 1.0, 0.5, atol=1e-3)  # pinned half-way (they interact weakly)
    assert np.allclose(np.diff(zeros), ny / 2, atol=1e-3)
    # The discrete equilibrium is not the continuum tanh profile: the test
    # sees the difference.
    y = np.arange(ny)
    psi_eq, l = np.sqrt(-a / b), np.sqrt(-2 * kappa / a)
    z0 = zeros[0]
    cont = psi_eq * (np.tanh((y - z0) / l) - np.tanh((y - z0 - ny / 2) / l) - 1)
    assert np.abs(ref - cont).max() > 1e-4
