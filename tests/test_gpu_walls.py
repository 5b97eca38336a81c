"""GPU parity with walls across the last axis (the closing remark of Sec. V.B:
the FV scheme admits walls and shear boundaries): halfway bounce-back of the
LB populations with the moving-wall term, and SMOL stencils without the
links that cross a wall.  Element by element against the oracle on the same
Philox stream (FP64 within 1e-12, FP32-deviation within 1e-5), on D2Q9,
D3Q15 and D3Q19, one- and two-phase, static and sliding walls, Euler, Heun
and RK4; the Couette profile; conservation of mass and psi."""
import numpy as np
import pytest

from tests import harness as H

pytestmark = pytest.mark.gpu

SHAPES = {H.D2Q9: (37, 22, 1), H.D3Q15: (19, 14, 11), H.D3Q19: (21, 13, 12)}
SLIDE = ((0.02, -0.01, 0.0), (-0.015, 0.01, 0.0))


def _slide(lattice):
    if lattice == H.D2Q9:  # 2-D walls are normal to y: they slide along x
        return ((0.02, 0.0, 0.0), (-0.015, 0.0, 0.0))
    return SLIDE


def _check(c, nsteps):
    from paper_1104_0078_amd import lbl
    print("walls case:", c, "steps", nsteps, flush=True)
    ini = lbl.make_init(kind=c["init"], psi_std=c["psi_std"])
    with lbl.Sim(H.lbl_params(c), ini) as sim:
        sim.step(nsteps)
        f_gpu, psi_gpu = sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI)
    f_ref, psi_ref = H.oracle_run(c, nsteps)
    ef, ep = H.rel_err(f_gpu, f_ref), H.rel_err(psi_gpu, psi_ref)
    print("  rel err populations %.3e psi %.3e" % (ef, ep), flush=True)
    tol = H.TOL[c["precision"]]
    assert ef <= tol and ep <= tol


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q15, H.D3Q19])
@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
@pytest.mark.parametrize("two_phase", [False, True])
@pytest.mark.parametrize("sliding", [False, True])
def test_walls_parity(lattice, precision, two_phase, sliding):
    kw = dict(a=-0.04, b=0.04, kappa=0.05, init=1) if two_phase else {}
    uw = _slide(lattice) if sliding else ((0, 0, 0), (0, 0, 0))
    c = H.config(lattice=lattice, smol=H.FV, precision=precision, shape=SHAPES[lattice],
                 kT=1e-4, walls=1, u_wall=uw, **kw)
    _check(c, 20)


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q19])
@pytest.mark.parametrize("rk", [1, 4])
def test_walls_parity_euler_rk4(lattice, rk):
    c = H.config(lattice=lattice, smol=H.FV, rk=rk, shape=SHAPES[lattice], a=-0.04, b=0.04,
                 kappa=0.05, init=1, kT=1e-5, walls=1, u_wall=_slide(lattice))
    _check(c, 20)


@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_walls_window_d3q19(precision):
    """The 100-step acceptance window with sliding walls, two-phase."""
    c = H.config(lattice=H.D3Q19, smol=H.FV, precision=precision, shape=SHAPES[H.D3Q19],
                 a=-0.04, b=0.04, kappa=0.05, init=1, kT=1e-5, walls=1, u_wall=SLIDE)
    _check(c, 100)


@pytest.mark.parametrize("coupling", [H.SMOL_ONLY, H.LB_ONLY])
def test_walls_partial_couplings(coupling):
    c = H.config(lattice=H.D3Q19, smol=H.FV, coupling=coupling, shape=SHAPES[H.D3Q19],
                 kT=1e-4, walls=1, u_wall=SLIDE, u_imposed=(0.02, -0.01, 0.0))
    _check(c, 15)


@pytest.mark.parametrize("lattice,shape", [(H.D2Q9, (8, 12, 1)), (H.D3Q19, (6, 5, 12))])
def test_walls_couette_profile(lattice, shape):
    """Walls sliding at -U and +U with every mode relaxed at the shear rate:
    the exact linear profile u_x = -U + 2U (h + 1/2)/L."""
    from paper_1104_0078_amd import lbl
    U = 0.02
    ws = 1 / (0.5 + 3 * 0.1)
    c = H.config(lattice=lattice, smol=H.FV, coupling=H.LB_ONLY, shape=shape, kT=0.0,
                 eta=0.1, omega_bulk=ws, omega_ghost=ws, walls=1,
                 u_wall=((-U, 0, 0), (U, 0, 0)), psi_std=0.0)
    with lbl.Sim(H.lbl_params(c), lbl.make_init(psi_std=0.0)) as sim:
        sim.step(6000)
        u = sim.observe(lbl.LBL_OBS_U)
    N = shape[0] * shape[1] * shape[2]
    d = 2 if lattice == H.D2Q9 else 3
    L = shape[d - 1]
    h = np.arange(N) // (shape[0] * (shape[1] if d == 3 else 1))
    want = -U + 2 * U * (h + 0.5) / L
    err = np.abs(u[0] - want).max()
    print("  Couette: max |u_x - linear| = %.2e" % err, flush=True)
    assert err < 1e-10 and np.abs(u[1:]).max() < 1e-12


@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_walls_conservation(precision):
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=H.D3Q19, smol=H.FV, precision=precision, shape=(24, 20, 18),
                 a=-0.04, b=0.04, kappa=0.05, init=1, kT=1e-5, walls=1, u_wall=SLIDE)
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3)) as sim:
        t0 = sim.observe(lbl.LBL_OBS_TOTALS)
        sim.step(200)
        t1 = sim.observe(lbl.LBL_OBS_TOTALS)
    tol = 1e-13 if precision == H.FP64 else 1e-6
    assert abs(t1[0] - t0[0]) <= tol * t0[5]
    assert abs(t1[4] - t0[4]) <= tol * t0[9]


def test_walls_schedules_do_not_change_results():
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=H.D3Q19, smol=H.FV, shape=(70, 21, 13), init=1, a=-0.04, b=0.04,
                 kappa=0.05, walls=1, u_wall=SLIDE)
    out = []
    # z-chunks of 4 and 5 planes put chunk edges next to both walls (nz = 13)
    for w, swz, zc, ov in ((64, 0, 0, 0), (32, 1, 4, 1), (256, 3, 5, 2), (128, 2, 13, 0),
                           (64, 0, 0, 3), (128, 2, 4, 3), (32, 0, 5, 3)):
        with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3)) as sim:
            sim.set_schedule(lb_width=w, xcd_swizzle=swz, zc=zc, overlap=ov)
            sim.step(6)
            out.append((sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI)))
    for f, p in out[1:]:
        np.testing.assert_array_equal(f, out[0][0])
        np.testing.assert_array_equal(p, out[0][1])


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q19])
def test_walls_user_init_roundtrip(lattice):
    """A user state with sliding walls: observed back bit for bit (the stored
    post-collision layout inverts the bounce-back at the wall layers), then
    10 steps against the oracle from the same state."""
    from paper_1104_0078_amd import lbl
    import oracle as O
    from tests import inputs
    c = H.config(lattice=lattice, smol=H.FV, shape=SHAPES[lattice], kT=1e-5, a=-0.04, b=0.04,
                 kappa=0.05, walls=1, u_wall=_slide(lattice))
    p = H.oracle_params(c)
    _, w = O.velocities(lattice)
    N = O.nsites(p)
    f0 = inputs.perturbed_populations(w, N, 0.05, seed=13)
    psi0 = inputs.random_field(N, 0.5, seed=14)
    print("walls user-init case:", c["shape"], flush=True)
    ini = lbl.make_init(kind=lbl.LBL_INIT_USER, f0=f0, psi0=psi0)
    with lbl.Sim(H.lbl_params(c), ini) as sim:
        np.testing.assert_array_equal(sim.observe(lbl.LBL_OBS_PSI), psi0)
        back = sim.observe(lbl.LBL_OBS_POP)
        # one rounding of (f + t) - t at the wall layers, exact elsewhere
        assert np.abs(back - f0).max() <= 4e-16 * np.abs(f0).max()
        sim.step(10)
        f_gpu, psi_gpu = sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI)
    f, psi = f0.copy(), psi0.copy()
    O.run(p, f, psi, 0, 10)
    ef, ep = H.rel_err(f_gpu, f), H.rel_err(psi_gpu, psi)
    print("  rel err populations %.3e psi %.3e" % (ef, ep), flush=True)
    assert ef <= 1e-12 and ep <= 1e-12


def test_walls_static_entry_point_matches_allocating_path():
    """lbl_step_static with sliding walls: equal to lbl_create + lbl_step
    from the same state."""
    import torch
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=H.D3Q19, smol=H.FV, shape=(20, 14, 12), a=-0.04, b=0.04, kappa=0.05,
                 init=1, kT=1e-5, walls=1, u_wall=SLIDE)
    print("walls static case:", c["shape"], flush=True)
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3)) as sim:
        sim.step(3)
        f3, p3 = sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI)
        sim.step(5)
        f8, p8 = sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI)
    pop = torch.from_numpy(np.ascontiguousarray(f3).reshape(-1)).cuda()
    psi = torch.from_numpy(np.ascontiguousarray(p3)).cuda()
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    rc = lbl.lbl_step_static(H.lbl_params(c), stream.cuda_stream, 3, 5, pop.data_ptr(),
                             psi.data_ptr())
    assert rc == lbl.LBL_OK, lbl.lbl_last_error(None)
    stream.synchronize()
    f_s, p_s = pop.cpu().numpy().reshape(f8.shape), psi.cpu().numpy()
    # the re-entry passes the state through the observed (streamed) form,
    # which rounds (f + t) - t once at the wall layers
    assert H.rel_err(f_s, f8) <= 1e-14 and H.rel_err(p_s, p8) <= 1e-14


@pytest.mark.parametrize("lattice,shape", [(H.D2Q9, (13, 17, 1)), (H.D3Q19, (7, 7, 11))])
@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_walls_fluctuation_profile(lattice, shape, precision):
    """Thermal fluctuations between walls: the SMOL alone (B = 0, no flow,
    A = 0.04, K = 0.05, M = 0.1, kT = 1e-5) from psi = 0.  Per layer parallel
    to the walls, the variance of psi - mean(psi) over 6000 samples (every
    25 steps after 20 000) against the exact stationary covariance of the
    discrete frozen-noise Heun scheme built from the oracle's operators with
    walls (tests/theory.stationary_covariance, pinned to the closed form on
    periodic lattices and to the Boltzmann limit with walls).  The layers
    next to the walls fluctuate ~30% more than the bulk; each layer within
    max(2%, 3 SE), SE from 30 batch means."""
    from paper_1104_0078_amd import lbl
    from tests import theory as T
    c = H.config(lattice=lattice, smol=H.FV, coupling=H.SMOL_ONLY, precision=precision,
                 shape=shape, a=0.04, b=0.0, kappa=0.05, M=0.1, kT=1e-5, walls=1, psi_std=0.0)
    p = H.oracle_params(c)
    L, Hm, Dv = T.smol_linear_operators(p)
    C = T.stationary_covariance(L, Hm, Dv, 1e-5, 0.1)
    d = 2 if lattice == H.D2Q9 else 3
    nl = shape[d - 1]
    want = np.diag(C).reshape(nl, -1).mean(axis=1)
    print("walls fluctuation case:", lattice, shape, "precision", precision, flush=True)
    nsamp, every = 6000, 25
    series = np.empty((nsamp, nl))
    with lbl.Sim(H.lbl_params(c), lbl.make_init(psi_std=0.0)) as sim:
        sim.step(20000)
        for k in range(nsamp):
            sim.step(every)
            psi = sim.observe(lbl.LBL_OBS_PSI)
            series[k] = ((psi - psi.mean()) ** 2).reshape(nl, -1).mean(axis=1)
    nb = 30
    bm = series[:nsamp // nb * nb].reshape(nb, -1, nl).mean(axis=1)
    got, se = bm.mean(axis=0), bm.std(axis=0, ddof=1) / np.sqrt(nb)
    ratio, rse = got / want, se / want
    print("  layer variance / prediction:", np.round(ratio, 4).tolist(), flush=True)
    print("  prediction wall / middle layer: %.4f, measured %.4f" % (
        want[0] / want[nl // 2], got[0] / got[nl // 2]), flush=True)
    assert np.all(np.abs(ratio - 1) <= np.maximum(0.02, 3 * rse))
    assert want[0] > 1.2 * want[nl // 2]


@pytest.mark.parametrize("lattice,shape", [(H.D2Q9, (16, 24, 1)), (H.D3Q19, (8, 8, 16))])
def test_walls_lb_equipartition(lattice, shape):
    """The fluctuating fluid between static walls (LB alone, kT = 1e-5, from
    rest): per layer and velocity component, <u_a^2> rho0 / kT = 1 within
    max(2%, 3 SE) (4000 samples every 20 steps after 5000; SE from 20 batch
    means).  Halfway bounce-back permutes a site's populations between
    directions of equal weight, so it keeps the equilibrium fluctuations,
    including those of the layers next to the walls (measured 0.99-1.01)."""
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=lattice, smol=H.FV, coupling=H.LB_ONLY, shape=shape, kT=1e-5, eta=0.1,
                 walls=1, psi_std=0.0)
    d = 2 if lattice == H.D2Q9 else 3
    nl = shape[d - 1]
    nsamp = 4000
    series = np.empty((nsamp, d, nl))
    print("walls equipartition case:", lattice, shape, flush=True)
    with lbl.Sim(H.lbl_params(c), lbl.make_init(psi_std=0.0)) as sim:
        sim.step(5000)
        for k in range(nsamp):
            sim.step(20)
            u = sim.observe(lbl.LBL_OBS_U).reshape(d, -1)
            series[k] = (u ** 2).reshape(d, nl, -1).mean(axis=2) / 1e-5
    nb = 20
    bm = series.reshape(nb, -1, d, nl).mean(axis=1)
    got, se = bm.mean(axis=0), bm.std(axis=0, ddof=1) / np.sqrt(nb)
    print("  <u_a^2> rho0/kT per layer:", np.round(got, 3).tolist(), flush=True)
    assert np.all(np.abs(got - 1) <= np.maximum(0.02, 3 * se))
