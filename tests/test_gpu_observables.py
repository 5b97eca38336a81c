"""GPU parity of the on-device Fourier observables and of the non-finite
trap: the sampled axis structure factors S_a(k) and velocity spectra
U_ab(k), and the means of their squares, against the oracle's axis spectra of
the same trajectory; the instantaneous psi(k) against numpy's FFT of the
oracle's field."""
import numpy as np
import pytest

import oracle as O
from tests import harness as H

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lattice,shape,smol", [(H.D2Q9, (40, 28, 1), H.FD),
                                                (H.D3Q19, (20, 12, 10), H.FV),
                                                (H.D3Q15, (12, 14, 10), H.FV)])
@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_sampled_spectra_match_oracle(lattice, shape, smol, precision):
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=lattice, smol=smol, precision=precision, shape=shape, kT=1e-4)
    print("sampling case", c, flush=True)
    every, nsteps = 2, 6
    with lbl.Sim(H.lbl_params(c, sample_every=every), lbl.make_init(psi_std=1e-2)) as sim:
        sim.step(nsteps)
        sk = sim.observe(lbl.LBL_OBS_SK_AXES)
        uk = sim.observe(lbl.LBL_OBS_UK_AXES)
        sk2 = sim.observe(lbl.LBL_OBS_SK2_AXES)
        uk2 = sim.observe(lbl.LBL_OBS_UK2_AXES)
        assert sim.observe(lbl.LBL_OBS_NSAMPLES) == nsteps // every
        psik = sim.observe(lbl.LBL_OBS_PSIK_AXES)
    p = H.oracle_params(c)
    f, psi = O.init(p, 0, 1e-2)
    d = O.d_of(p)
    L = max(shape)
    sk_ref = np.zeros((d, L))
    uk_ref = np.zeros((d, d, L))
    sk2_ref = np.zeros((d, L))
    uk2_ref = np.zeros((d, d, L))
    for n in range(nsteps):
        u = O.velocity(p, f, O.force(p, psi))
        O.step(p, f, psi, n)
        if (n + 1) % every == 0:
            s_ = O.axis_spectrum(p, psi, L)
            sk_ref += s_
            sk2_ref += s_ ** 2
            for b in range(d):
                u_ = O.axis_spectrum(p, u[b], L)
                uk_ref[:, b, :] += u_
                uk2_ref[:, b, :] += u_ ** 2
    ns = nsteps // every
    sk_ref, uk_ref, sk2_ref, uk2_ref = sk_ref / ns, uk_ref / ns, sk2_ref / ns, uk2_ref / ns
    tol = 1e-11 if precision == H.FP64 else 2e-5
    assert H.rel_err(sk, sk_ref) < tol
    assert H.rel_err(uk, uk_ref) < tol
    assert H.rel_err(sk2, sk2_ref) < 2 * tol
    assert H.rel_err(uk2, uk2_ref) < 2 * tol
    grid = psi.reshape(shape[::-1] if d == 3 else shape[1::-1])
    F = np.fft.fftn(grid)  # axes (z,) y, x
    ref = [F[0, :], F[:, 0]] if d == 2 else [F[0, 0, :], F[0, :, 0], F[:, 0, 0]]
    for a in range(d):
        n_a = len(ref[a])
        np.testing.assert_allclose(psik[a][:n_a], ref[a],
                                   atol=tol * 10 * np.abs(ref[a]).max())


def test_nonfinite_state_is_reported():
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=H.D2Q9, smol=H.FD, shape=(32, 32, 1))
    p = H.oracle_params(c)
    f0, psi0 = O.init(p, 0, 1e-3)
    psi0[100] = np.nan
    ini = lbl.make_init(kind=lbl.LBL_INIT_USER, f0=f0, psi0=psi0)
    with lbl.Sim(H.lbl_params(c, sample_every=1), ini) as sim:
        sim.step(2)
        with pytest.raises(lbl.LblError) as e:
            sim.observe(lbl.LBL_OBS_PSI)
        assert e.value.code == lbl.LBL_E_NONFINITE


@pytest.mark.parametrize("lattice,shape,precision", [(H.D2Q9, (21, 13, 1), H.FP64),
                                                     (H.D3Q19, (12, 9, 7), H.FP64),
                                                     (H.D3Q15, (10, 8, 6), H.FP32DEV)])
def test_full_k_structure_factor(lattice, shape, precision):
    """LBL_OBS_SK_FULL (hipFFT of psi at every sample) against numpy's real
    FFT of the same psi snapshots; on the axes it equals SK_AXES."""
    from paper_1104_0078_amd import lbl
    nx, ny, nz = shape
    N = nx * ny * nz
    c = H.config(lattice=lattice, smol=H.FV, precision=precision, shape=shape, kT=1e-4,
                 a=-0.04, b=0.04, init=1)
    params = H.lbl_params(c, sample_every=1)
    params.sample_full_k = 1
    acc = np.zeros((nz, ny, nx // 2 + 1))
    with lbl.Sim(params, lbl.make_init(kind=1, psi_std=1e-2)) as sim:
        for _ in range(4):
            sim.step(1)
            psi = sim.observe(lbl.LBL_OBS_PSI).reshape(nz, ny, nx)
            acc += np.abs(np.fft.rfftn(psi)) ** 2 / N
        sk = sim.observe(lbl.LBL_OBS_SK_FULL)
        axes = sim.observe(lbl.LBL_OBS_SK_AXES)
        assert sim.observe(lbl.LBL_OBS_NSAMPLES) == 4
    acc /= 4
    tol = 1e-12 if precision == H.FP64 else 2e-5
    np.testing.assert_allclose(sk, acc, rtol=tol, atol=tol * acc.max())
    m = np.arange(nx // 2 + 1)
    np.testing.assert_allclose(sk[0, 0, m], axes[0, m], rtol=tol, atol=tol * acc.max())
    c2 = H.config(lattice=H.D2Q9, smol=H.FD, shape=(8, 8, 1))
    with lbl.Sim(H.lbl_params(c2, sample_every=1), lbl.make_init()) as sim:
        with pytest.raises(lbl.LblError):
            sim.observe(lbl.LBL_OBS_SK_FULL)


@pytest.mark.parametrize("lattice,shape", [(H.D2Q9, (70, 48, 1)), (H.D3Q19, (21, 13, 24)),
                                           (H.D3Q15, (19, 14, 16))])
@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_interface_heights(lattice, shape, precision):
    """LBL_OBS_HEIGHTS (Sec. VI.C) equals the oracle's heights of the same psi
    (the observed PSI), and the oracle's heights of its own trajectory within
    the parity bar scaled by the interface slope."""
    from paper_1104_0078_amd import lbl
    import oracle as O
    c = H.config(lattice=lattice, smol=H.FV, precision=precision, shape=shape, a=-0.04,
                 b=0.04, kappa=0.05, init=1, kT=1e-4, psi_std=1e-2)
    p = H.oracle_params(c)
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-2)) as sim:
        sim.step(12)
        h = sim.observe(lbl.LBL_OBS_HEIGHTS).reshape(2, -1)
        psi = sim.observe(lbl.LBL_OBS_PSI)
    assert np.isfinite(h).all()
    np.testing.assert_allclose(h, O.heights(p, psi), rtol=0, atol=1e-12)
    _, psi_ref = H.oracle_run(c, 12)
    L = shape[2] if lattice != H.D2Q9 else shape[1]
    assert np.abs(h[0] - L / 4).max() < 2 and np.abs(h[1] - 3 * L / 4).max() < 2
    tol = 1e-10 if precision == H.FP64 else 1e-3
    np.testing.assert_allclose(h, O.heights(p, psi_ref), rtol=0, atol=tol)
