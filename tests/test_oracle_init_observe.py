"""Pins of the oracle's initial states and observables.

* Two flat interfaces: psi = psi_eq [tanh((h - L/4)/l) - tanh((h - 3L/4)/l) - 1]
  with psi_eq = sqrt(-A/B) and l = sqrt(-2K/A) (Eqs. tanh, intthick with A < 0).
* The rest state is the second-order equilibrium: density rho0, velocity U.
* Axis structure factors equal numpy's FFT of the field along the axes.
* Totals equal direct sums.
"""
import numpy as np
import pytest

import oracle as O


def test_tanh_two_interfaces():
    p = O.make_params(lattice=O.D3Q19, shape=(4, 3, 40), a=-0.04, b=0.04, kappa=0.05)
    f, psi = O.init(p, 1, 0.0)
    h = np.arange(O.nsites(p)) // (p.nx * p.ny)
    l = np.sqrt(2 * 0.05 / 0.04)
    expect = np.tanh((h - 10) / l) - np.tanh((h - 30) / l) - 1
    np.testing.assert_allclose(psi, expect, atol=1e-15)
    assert abs(l - 1.5811388300841898) < 1e-15
    p2 = O.make_params(lattice=O.D2Q9, shape=(5, 32, 1), a=-0.09, b=0.04, kappa=0.05)
    _, psi2 = O.init(p2, 1, 0.0)
    h2 = (np.arange(O.nsites(p2)) // p2.nx) % p2.ny
    l2 = np.sqrt(2 * 0.05 / 0.09)
    np.testing.assert_allclose(psi2, 1.5 * (np.tanh((h2 - 8) / l2) - np.tanh((h2 - 24) / l2) - 1),
                               atol=1e-15)
    with pytest.raises(ValueError):
        O.init(O.make_params(a=0.04), 1, 0.0)


def test_rest_state_and_noise():
    p = O.make_params(lattice=O.D2Q9, shape=(64, 64, 1), rho0=1.2)
    f, psi = O.init(p, 0, 1e-3, boost=(0.01, -0.02))
    c, w = O.velocities(O.D2Q9)
    rho = f.sum(0)
    j = c[:, :2].T.astype(float) @ f
    np.testing.assert_allclose(rho, 1.2, rtol=1e-15)
    np.testing.assert_allclose(j[0], 1.2 * 0.01, rtol=1e-13)
    np.testing.assert_allclose(j[1], -1.2 * 0.02, rtol=1e-13)
    assert abs(psi.std() / 1e-3 - 1) < 0.05
    assert abs(psi.mean()) < 5e-3 / 64
    for s in (0, 17, 4095):
        assert psi[s] == 1e-3 * O.normal(p.seed, s, 0, O.TAG_INIT, 0)


def test_axis_spectrum_and_totals():
    rng = np.random.default_rng(5)
    p = O.make_params(lattice=O.D3Q19, shape=(7, 5, 6))
    N = O.nsites(p)
    field = rng.standard_normal(N)
    S = O.axis_spectrum(p, field)
    F = np.fft.fftn(field.reshape(6, 5, 7))
    np.testing.assert_allclose(S[0][:7], np.abs(F[0, 0, :]) ** 2 / N, rtol=1e-12)
    np.testing.assert_allclose(S[1][:5], np.abs(F[0, :, 0]) ** 2 / N, rtol=1e-12)
    np.testing.assert_allclose(S[2][:6], np.abs(F[:, 0, 0]) ** 2 / N, rtol=1e-12)
    f = rng.standard_normal((19, N))
    t = O.totals(p, f, field)
    c, _ = O.velocities(O.D3Q19)
    j = c.T.astype(float) @ f
    np.testing.assert_allclose(t[0], f.sum(), rtol=1e-12)
    np.testing.assert_allclose(t[1:4], j.sum(1), rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(t[4], field.sum(), rtol=1e-12)
    np.testing.assert_allclose(t[5], np.abs(f.sum(0)).sum(), rtol=1e-12)
    np.testing.assert_allclose(t[6:9], np.abs(j).sum(1), rtol=1e-12)
    np.testing.assert_allclose(t[9], np.abs(field).sum(), rtol=1e-12)


@pytest.mark.parametrize("lattice,shape", [(O.D2Q9, (12, 40, 1)), (O.D3Q19, (6, 5, 48))])
def test_interface_heights_closed_form(lattice, shape):
    """Heights of the two interfaces (Sec. VI.C, zero crossing by linear
    interpolation): on columns whose profile is linear through a chosen
    crossing z* (clipped to +-1 away from it), the height is z* to rounding;
    a column without a sign change in a window gives NaN; the flat two-phase
    initial state has its interfaces at L/4 and 3L/4 exactly."""
    p = O.make_params(lattice=lattice, shape=shape, a=-0.04, b=0.04, kappa=0.05)
    d = O.d_of(p)
    L = shape[2] if d == 3 else shape[1]
    C = shape[0] * shape[1] if d == 3 else shape[0]
    rng = np.random.default_rng(3)
    zlo = rng.uniform(L / 8 + 1, 3 * L / 8 - 1, C)
    zhi = rng.uniform(5 * L / 8 + 1, 7 * L / 8 - 1, C)
    z = np.arange(L)[:, None]
    col = np.where(z < L // 2, np.clip(z - zlo, -1, 1), np.clip(zhi - z, -1, 1))
    col[:, 0] = 0.5  # no crossing anywhere in this column
    psi = np.ascontiguousarray(col.reshape(-1))  # site = c + C * z
    h = O.heights(p, psi)
    np.testing.assert_allclose(h[0, 1:], zlo[1:], rtol=0, atol=1e-13)
    np.testing.assert_allclose(h[1, 1:], zhi[1:], rtol=0, atol=1e-13)
    assert np.isnan(h[:, 0]).all()
    _, psi0 = O.init(p, 1, 0.0)
    h0 = O.heights(p, psi0)
    np.testing.assert_allclose(h0[0], L / 4, atol=1e-12)
    np.testing.assert_allclose(h0[1], 3 * L / 4, atol=1e-12)


@pytest.mark.parametrize("l", [1.58, 2.83])
def test_height_estimator_gain(l):
    """The gain of the linear-interpolation heights on a tanh profile (the
    correction the capillary tests apply) against finite differences of the
    oracle's own estimator: columns psi = tanh((z - h)/l) with the lower
    interface at h = 12 + delta, moved by +-1e-6."""
    from tests import theory as T
    L = 48
    # offsets inside the cell (at delta = 0 the gain has a kink, where a
    # central difference is off by O(eps)); one column each
    delta = np.append(np.linspace(0.0125, 0.9875, 40), [0.5, 1e-3])
    p = O.make_params(lattice=O.D2Q9, shape=(delta.size, L, 1), a=-0.04, b=0.04, kappa=0.05)
    z = np.arange(L)[:, None]
    eps = 1e-6

    def est(h):
        col = np.where(z < L // 2, np.tanh((z - h[None, :]) / l), np.tanh((36.0 - z) / l))
        return O.heights(p, np.ascontiguousarray(col.reshape(-1)))[0]

    hc = 12.0 + delta
    g = (est(hc + eps) - est(hc - eps)) / (2 * eps)
    np.testing.assert_allclose(g, T.interp_gain(delta, l), rtol=1e-7)
    # on a site and half-way between sites; mean over the offsets
    assert abs(T.interp_gain(0.0, l) - 1 / (l * np.tanh(1 / l))) < 1e-15
    dd = (np.arange(100000) + 0.5) / 100000
    assert abs(T.interp_gain(dd, l).mean() - 1) < 1e-9
