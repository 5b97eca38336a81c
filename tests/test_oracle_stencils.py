"""Pins of the oracle's discrete operators: each applied to a plane wave
e^{i q.x} must return its closed-form lattice symbol times the wave.

Closed forms:
  * 3-D Shinozaki-Oono Laplacian: the paper's Eq. (solapft), App. A.
  * 2-D Laplacian (reading; the paper gives 3-D only): cos qx + cos qy + cos qx cos qy - 3.
  * FD gradient / divergence (Sec. IV, Sec. V.A central differences): i sin q_a.
  * FV gradient Gamma(q) = (1/c_s^2) sum_i w_i c_i e^{i q.c_i} (Eq. fvgrad), which for
    D3Q19 is (i/3) sin q_x (1 + cos q_y + cos q_z) and for D2Q9 (i/3) sin q_x (2 + cos q_y),
    and the FV Laplacian Gamma.Gamma.
The last test checks the FV normalisation reading against the paper's own printed
D3Q15 symbol, Eq. (fvlapft).
"""
import itertools

import numpy as np
import pytest

import oracle as O


def _coords(p):
    N = O.nsites(p)
    s = np.arange(N)
    return s % p.nx, (s // p.nx) % p.ny, s // (p.nx * p.ny)


def _wave(p, k):
    x, y, z = _coords(p)
    q = 2 * np.pi * np.array([k[0] / p.nx, k[1] / p.ny, k[2] / p.nz])
    ph = q[0] * x + q[1] * y + q[2] * z
    return q, np.cos(ph), np.sin(ph), np.exp(1j * ph)


def _apply_scalar(fn, p, k):
    q, c, s, e = _wave(p, k)
    out = fn(p, c) + 1j * fn(p, s)
    return q, out, e


def _wavevectors(p, n=25, seed=0):
    rng = np.random.default_rng(seed)
    ks = [(0, 0, 0), (p.nx // 2, 0, 0), (1, 1, 1 if p.nz > 1 else 0)]
    for _ in range(n):
        ks.append((int(rng.integers(p.nx)), int(rng.integers(p.ny)),
                   int(rng.integers(p.nz)) if p.nz > 1 else 0))
    return ks


def so3(q):
    cx, cy, cz = np.cos(q)
    return (12 * (cx + cy + cz) + 12 * (cx * cy + cx * cz + cy * cz) + 8 * cx * cy * cz - 80) / 22


def so2(q):
    cx, cy = np.cos(q[:2])
    return cx + cy + cx * cy - 3


def gamma_fv(q, lattice):
    s, c = np.sin(q), np.cos(q)
    if lattice == O.D3Q19:
        return 1j / 3 * np.array([s[0] * (1 + c[1] + c[2]), s[1] * (1 + c[0] + c[2]),
                                  s[2] * (1 + c[0] + c[1])])
    if lattice == O.D3Q15:
        return 1j / 3 * np.array([s[0] * (2 + c[1] * c[2]), s[1] * (2 + c[0] * c[2]),
                                  s[2] * (2 + c[0] * c[1])])
    return 1j / 3 * np.array([s[0] * (2 + c[1]), s[1] * (2 + c[0])])


CASES = [(O.D2Q9, (12, 10, 1)), (O.D3Q15, (7, 6, 5)), (O.D3Q19, (8, 6, 5))]


@pytest.mark.parametrize("lattice,shape", CASES)
def test_laplacian_symbol(lattice, shape):
    p = O.make_params(lattice=lattice, shape=shape)
    for k in _wavevectors(p):
        q, out, e = _apply_scalar(O.laplacian, p, k)
        sym = so3(q) if lattice != O.D2Q9 else so2(q)
        np.testing.assert_allclose(out, sym * e, atol=1e-14)
        # the small-q limit is -q^2 for every admissible stencil (Sec. III)
    p2 = O.make_params(lattice=lattice, shape=(64, 64, 64 if lattice != O.D2Q9 else 1))
    q = 2 * np.pi * np.array([1, 2, 1 if lattice != O.D2Q9 else 0]) / 64
    sym = so3(q) if lattice != O.D2Q9 else so2(q)
    assert abs(sym + q @ q) < 0.01 * (q @ q)


@pytest.mark.parametrize("lattice,shape", CASES)
@pytest.mark.parametrize("smol", [O.FD, O.FV])
def test_gradient_and_divergence_symbols(lattice, shape, smol):
    p = O.make_params(lattice=lattice, smol=smol, shape=shape)
    d = O.d_of(p)
    for k in _wavevectors(p):
        q, c, s, e = _wave(p, k)
        sym = 1j * np.sin(q[:d]) if smol == O.FD else gamma_fv(q, lattice)
        g = O.gradient(p, c) + 1j * O.gradient(p, s)
        for a in range(d):
            np.testing.assert_allclose(g[a], sym[a] * e, atol=1e-14)
            v = np.zeros((d, O.nsites(p)))
            v[a] = c
            vs = np.zeros((d, O.nsites(p)))
            vs[a] = s
            div = O.divergence(p, v) + 1j * O.divergence(p, vs)
            np.testing.assert_allclose(div, sym[a] * e, atol=1e-14)


@pytest.mark.parametrize("lattice,shape", CASES)
def test_fv_laplacian_symbol(lattice, shape):
    p = O.make_params(lattice=lattice, smol=O.FV, shape=shape)
    for k in _wavevectors(p):
        q, c, s, e = _wave(p, k)
        lc = O.divergence(p, O.gradient(p, c))
        ls = O.divergence(p, O.gradient(p, s))
        sn, cs = np.sin(q), np.cos(q)
        if lattice == O.D3Q19:
            sym = -(sn[0] ** 2 * (1 + cs[1] + cs[2]) ** 2 + sn[1] ** 2 * (1 + cs[0] + cs[2]) ** 2
                    + sn[2] ** 2 * (1 + cs[0] + cs[1]) ** 2) / 9
        elif lattice == O.D3Q15:
            # The paper's own FV Laplacian of D3Q15, Eq. (fvlapft), written out.
            sym = -((2 * sn[0] + sn[0] * cs[1] * cs[2]) ** 2
                    + (2 * sn[1] + sn[1] * cs[0] * cs[2]) ** 2
                    + (2 * sn[2] + sn[2] * cs[0] * cs[1]) ** 2) / 9
        else:
            sym = -(sn[0] ** 2 * (2 + cs[1]) ** 2 + sn[1] ** 2 * (2 + cs[0]) ** 2) / 9
        np.testing.assert_allclose(lc + 1j * ls, sym * e, atol=1e-14)


def test_fv_normalisation_reproduces_paper_d3q15_symbol():
    # D3Q15 (the paper's lattice): rest 2/9, 6 axis links 1/9, 8 corners 1/72.
    vel = [(0, 0, 0)] + [v for v in itertools.product((-1, 0, 1), repeat=3)
                         if sum(map(abs, v)) in (1, 3)]
    w = [2 / 9] + [1 / 9 if sum(map(abs, v)) == 1 else 1 / 72 for v in vel[1:]]
    rng = np.random.default_rng(3)
    for q in rng.uniform(-np.pi, np.pi, size=(50, 3)):
        gam = 3 * sum(wi * np.array(v) * np.exp(1j * np.dot(q, v)) for wi, v in zip(w, vel))
        sx, sy, sz = np.sin(q)
        cx, cy, cz = np.cos(q)
        paper = -((2 * sx + sx * cy * cz) ** 2 + (2 * sy + sy * cx * cz) ** 2
                  + (2 * sz + sz * cx * cy) ** 2) / 9
        assert abs(np.dot(gam, gam) - paper) < 1e-14
