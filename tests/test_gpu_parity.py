"""GPU parity: the HIP sweep against the FP64 oracle, element by element, on
the same seeded inputs and the same Philox stream.

Sizes span several thread blocks and end in a ragged tail.  Bar: FP64 fields
within 1e-12 and FP32-deviation fields within 1e-5 of the oracle, relative to
the largest magnitude of the oracle field.
"""
import numpy as np
import pytest

from tests import harness as H

pytestmark = pytest.mark.gpu

SHAPES = {H.D2Q9: (70, 45, 1), H.D3Q15: (19, 14, 9), H.D3Q19: (21, 13, 11)}


def _gpu(c, nsteps, init=None):
    from paper_1104_0078_amd import lbl
    ini = init if init is not None else lbl.make_init(kind=c["init"], psi_std=c["psi_std"],
                                                      boost=c["boost"])
    with lbl.Sim(H.lbl_params(c), ini) as sim:
        sim.step(nsteps)
        return sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI), sim


def _check(c, nsteps, tol=None):
    print("parity case:", c, "steps", nsteps, flush=True)
    f_gpu, psi_gpu, _ = _gpu(c, nsteps)
    f_ref, psi_ref = H.oracle_run(c, nsteps)
    tol = tol if tol is not None else H.TOL[c["precision"]]
    ef, ep = H.rel_err(f_gpu, f_ref), H.rel_err(psi_gpu, psi_ref)
    print("  rel err populations %.3e psi %.3e" % (ef, ep), flush=True)
    assert ef <= tol and ep <= tol


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q15, H.D3Q19])
@pytest.mark.parametrize("smol", [H.FD, H.FV])
@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_coupled_one_phase(lattice, smol, precision):
    c = H.config(lattice=lattice, smol=smol, precision=precision, shape=SHAPES[lattice])
    _check(c, 20)


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q15, H.D3Q19])
@pytest.mark.parametrize("smol", [H.FD, H.FV])
def test_coupled_two_phase_tanh(lattice, smol):
    c = H.config(lattice=lattice, smol=smol, shape=SHAPES[lattice], a=-0.04, b=0.04,
                 kappa=0.05, init=1, kT=1e-5)
    _check(c, 20)


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q15, H.D3Q19])
@pytest.mark.parametrize("smol", [H.FD, H.FV])
@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
@pytest.mark.parametrize("rk", [1, 4])
def test_coupled_euler_and_rk4(lattice, smol, precision, rk):
    """Full coupling with Euler and RK4 stages, two-phase: the RK4 mid stages
    advect with the mean of u^n and the velocity of the streamed populations,
    and the RK4 accumulator carries the weighted stage sums."""
    c = H.config(lattice=lattice, smol=smol, precision=precision, rk=rk, shape=SHAPES[lattice],
                 a=-0.04, b=0.04, kappa=0.05, init=1, kT=1e-5)
    _check(c, 20)


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q19])
@pytest.mark.parametrize("rk", [1, 4])
def test_coupled_euler_and_rk4_one_phase(lattice, rk):
    c = H.config(lattice=lattice, smol=H.FV, rk=rk, shape=SHAPES[lattice], kT=1e-4)
    _check(c, 20)


# The acceptance window: GPU and oracle fields over the first 100 steps on the
# same Philox stream, FP64 within 1e-12 and FP32-deviation within 1e-5.
WINDOW = 100


@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_window_d2q9_fd_64(precision):
    """D2Q9 + FD on the 64 x 64 periodic lattice at tau_s = 0.8 (eta = 0.1),
    other rates 1, kT = 1e-5, M = 0.1, A = 0.04, B = 0.1, K = 0.05,
    psi0 = N(0, 1e-3), seed 1234."""
    c = H.config(lattice=H.D2Q9, smol=H.FD, precision=precision, shape=(64, 64, 1))
    _check(c, WINDOW)


@pytest.mark.parametrize("lattice", [H.D3Q15, H.D3Q19])
@pytest.mark.parametrize("two_phase", [False, True])
@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_window_3d_fv(lattice, two_phase, precision):
    kw = dict(a=-0.04, b=0.04, kappa=0.05, init=1) if two_phase else {}
    c = H.config(lattice=lattice, smol=H.FV, precision=precision, shape=SHAPES[lattice], **kw)
    _check(c, WINDOW)


@pytest.mark.parametrize("coupling", [H.SMOL_ONLY, H.LB_ONLY])
@pytest.mark.parametrize("rk", [1, 2, 4])
def test_partial_couplings_and_stages(coupling, rk):
    c = H.config(lattice=H.D2Q9, smol=H.FV, coupling=coupling, rk=rk, shape=(70, 45, 1),
                 u_imposed=(0.03, -0.02, 0.0), kT=1e-4)
    _check(c, 15)


@pytest.mark.parametrize("lattice", [H.D3Q15, H.D3Q19])
def test_mrt_rates_and_boost(lattice):
    c = H.config(lattice=lattice, smol=H.FV, shape=SHAPES[lattice], omega_bulk=1.3,
                 omega_ghost=0.8, eta=0.05, boost=(0.02, -0.01, 0.015), kT=1e-4)
    _check(c, 15)


def test_user_init_roundtrip():
    from paper_1104_0078_amd import lbl
    import oracle as O
    from tests import inputs
    c = H.config(lattice=H.D3Q19, smol=H.FD, shape=SHAPES[H.D3Q19], kT=1e-5)
    p = H.oracle_params(c)
    _, w = O.velocities(H.D3Q19)
    N = O.nsites(p)
    f0 = inputs.perturbed_populations(w, N, 0.05, seed=3)
    psi0 = inputs.random_field(N, 0.02, seed=4)
    ini = lbl.make_init(kind=lbl.LBL_INIT_USER, f0=f0, psi0=psi0)
    with lbl.Sim(H.lbl_params(c), ini) as sim:
        np.testing.assert_array_equal(sim.observe(lbl.LBL_OBS_POP), f0)
        np.testing.assert_array_equal(sim.observe(lbl.LBL_OBS_PSI), psi0)
        sim.step(10)
        f_gpu, psi_gpu = sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI)
    f, psi = f0.copy(), psi0.copy()
    O.run(p, f, psi, 0, 10)
    assert H.rel_err(f_gpu, f) < 1e-12 and H.rel_err(psi_gpu, psi) < 1e-12


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q19])
def test_observables_match_oracle(lattice):
    from paper_1104_0078_amd import lbl
    import oracle as O
    c = H.config(lattice=lattice, smol=H.FV, shape=SHAPES[lattice], a=-0.04, b=0.04, init=1)
    p = H.oracle_params(c)
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3)) as sim:
        sim.step(5)
        rho = sim.observe(lbl.LBL_OBS_RHO)
        u = sim.observe(lbl.LBL_OBS_U)
        tot = sim.observe(lbl.LBL_OBS_TOTALS)
        assert sim.observe(lbl.LBL_OBS_STEP) == 5
    f, psi = H.oracle_run(c, 5)
    assert H.rel_err(rho, f.sum(0)) < 1e-13
    uref = O.velocity(p, f, O.force(p, psi))
    assert H.rel_err(u, uref) < 1e-11
    tref = O.totals(p, f, psi)
    np.testing.assert_allclose(tot, tref, rtol=1e-12, atol=1e-13 * tref[5])


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q19])
@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_conservation_on_gpu(lattice, precision):
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=lattice, smol=H.FV, precision=precision, shape=SHAPES[lattice],
                 a=-0.04, b=0.04, init=1, kT=1e-5)
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3)) as sim:
        t0 = sim.observe(lbl.LBL_OBS_TOTALS)
        sim.step(100)
        t1 = sim.observe(lbl.LBL_OBS_TOTALS)
    tol = 1e-13 if precision == H.FP64 else 1e-6
    assert abs(t1[0] - t0[0]) <= tol * t0[5]
    assert abs(t1[4] - t0[4]) <= tol * t0[9]


@pytest.mark.parametrize("lattice,smol", [(H.D3Q19, H.FV), (H.D3Q15, H.FV), (H.D3Q19, H.FD),
                                          (H.D2Q9, H.FV), (H.D2Q9, H.FD)])
def test_default_schedule_draws_the_noise_in_the_velocity_pass(lattice, smol):
    """The default schedule draws the SMOL noise inside the velocity pass
    (overlap 3) on every lattice and variant."""
    overlap = 3
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=lattice, smol=smol, shape=SHAPES[lattice], init=0)
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=0, psi_std=1e-3)) as sim:
        assert sim.schedule()["overlap"] == overlap
        sim.set_schedule(lb_width=64, xcd_swizzle=0, zc=0, overlap=overlap)
        assert sim.schedule()["overlap"] == overlap


@pytest.mark.parametrize("smol", [H.FV, H.FD])
@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q19])
def test_schedule_does_not_change_results(lattice, smol):
    """Every launch schedule (LB block width, XCD-contiguous block order,
    planes per SMOL tile, first stage or SMOL noise on a second stream, SMOL
    noise drawn in the velocity pass) gives bitwise the same fields."""
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=lattice, smol=smol, shape=SHAPES[lattice], init=0)
    ini = lbl.make_init(kind=0, psi_std=1e-3)
    out = []
    for w, swz, zc, ov in ((64, 0, 0, 0), (256, 0, 0, 1), (128, 1, 0, 0), (32, 3, 3, 1),
                           (256, 2, 5, 0), (64, 0, 0, 2), (128, 3, 4, 2), (64, 0, 0, 3),
                           (128, 2, 3, 3)):
        with lbl.Sim(H.lbl_params(c), ini) as sim:
            sim.set_schedule(lb_width=w, xcd_swizzle=swz, zc=zc, overlap=ov)
            assert sim.schedule()["lb_width"] == w
            sim.step(7)
            out.append((sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI)))
    for f, p in out[1:]:
        np.testing.assert_array_equal(f, out[0][0])
        np.testing.assert_array_equal(p, out[0][1])


@pytest.mark.parametrize("lattice,shape", [(H.D2Q9, (4, 4, 1)), (H.D2Q9, (5, 33, 1)),
                                           (H.D3Q19, (4, 4, 4)), (H.D3Q19, (5, 7, 4)),
                                           (H.D3Q15, (4, 4, 4)), (H.D3Q15, (6, 5, 7)),
                                           (H.D3Q19, (33, 9, 5))])
@pytest.mark.parametrize("smol", [H.FD, H.FV])
@pytest.mark.parametrize("force_form", [0, 1])
def test_smallest_and_odd_lattices(lattice, shape, smol, force_form):
    """Sides at the minimum the ABI accepts (4, where every stencil halo
    wraps onto the lattice itself several times) and odd sides just past one
    tile, two-phase so that the nonlinear terms are exercised; with either
    force (the stress kernels' z-chunks then span the whole periodic axis)."""
    c = H.config(lattice=lattice, smol=smol, shape=shape, init=0, a=-0.04, b=0.04,
                 force_form=force_form)
    _check(c, 12)


def test_zero_steps_and_observe_before_stepping():
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=H.D2Q9, smol=H.FV, shape=(20, 12, 1), init=0)
    f_ref, psi_ref = H.oracle_run(c, 0)
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=0, psi_std=1e-3)) as sim:
        sim.step(0)
        assert sim.observe(lbl.LBL_OBS_STEP) == 0
        f = sim.observe(lbl.LBL_OBS_POP)
        psi = sim.observe(lbl.LBL_OBS_PSI)
    assert H.rel_err(f, f_ref) <= 1e-15 and H.rel_err(psi, psi_ref) <= 1e-15


@pytest.mark.parametrize("lattice,smol", [(H.D2Q9, H.FD), (H.D3Q19, H.FV)])
@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_resume_is_bitwise(lattice, smol, precision):
    """A simulation created from another one's POP and PSI at step n, with
    step0 = n, continues it bitwise (the noise counter carries on)."""
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=lattice, smol=smol, precision=precision, shape=SHAPES[lattice],
                 init=1, a=-0.04, b=0.04)
    ini = lbl.make_init(kind=1, psi_std=1e-3)
    with lbl.Sim(H.lbl_params(c), ini) as sim:
        sim.step(9)
        f9, p9 = sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI)
        sim.step(6)
        f15, p15 = sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI)
    res = lbl.make_init(kind=lbl.LBL_INIT_USER, f0=f9, psi0=p9, step0=9)
    with lbl.Sim(H.lbl_params(c), res) as sim:
        assert sim.observe(lbl.LBL_OBS_STEP) == 9
        sim.step(6)
        np.testing.assert_array_equal(sim.observe(lbl.LBL_OBS_POP), f15)
        np.testing.assert_array_equal(sim.observe(lbl.LBL_OBS_PSI), p15)


@pytest.mark.parametrize("lattice", [H.D3Q15, H.D3Q19])
@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
@pytest.mark.parametrize("force_form", [0, 1])
def test_wide_lattice_ragged_tiles(lattice, precision, force_form):
    """A lattice wider than the LB rows' 64-site blocks and the SMOL tiles,
    with ragged tiles in x (70 = 2 x 32 + 6) and y (21 = 2 x 8 + 5), and
    z-chunks of 8 and 1 planes in the stress-force kernel."""
    c = H.config(lattice=lattice, smol=H.FV, precision=precision, shape=(70, 21, 9), a=-0.04,
                 b=0.04, kappa=0.05, init=1, kT=1e-5, force_form=force_form)
    _check(c, 15)


@pytest.mark.parametrize("force_form", [0, 1])
def test_wide_lattice_schedules_do_not_change_results(force_form):
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=H.D3Q19, smol=H.FV, shape=(70, 21, 13), init=0, a=-0.04, b=0.04,
                 force_form=force_form)
    ini = lbl.make_init(kind=0, psi_std=1e-3)
    out = []
    for swz, zc, ov in ((0, 0, 0), (2, 4, 0), (0, 5, 1), (3, 13, 0), (1, 6, 2), (0, 0, 3),
                        (2, 4, 3), (1, 13, 3)):
        with lbl.Sim(H.lbl_params(c), ini) as sim:
            sim.set_schedule(lb_width=64, xcd_swizzle=swz, zc=zc, overlap=ov)
            sim.step(6)
            out.append((sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI)))
    for f, p in out[1:]:
        np.testing.assert_array_equal(f, out[0][0])
        np.testing.assert_array_equal(p, out[0][1])


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q15, H.D3Q19])
@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_fd_fourier_noise(lattice, precision):
    """FD noise built in Fourier space (hipFFT on the GPU, a plain DFT in the
    oracle) on lattices with odd sides, full coupling, two-phase."""
    c = H.config(lattice=lattice, smol=H.FD, precision=precision, shape=SHAPES[lattice],
                 a=-0.04, b=0.04, init=1, kT=1e-4, fd_noise=1)
    _check(c, 12)


def test_fd_fourier_noise_smol_only_rk4():
    c = H.config(lattice=H.D3Q19, smol=H.FD, coupling=H.SMOL_ONLY, rk=4, shape=(15, 12, 9),
                 kT=1e-4, u_imposed=(0.02, -0.01, 0.03), fd_noise=1)
    _check(c, 10)


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q15, H.D3Q19])
@pytest.mark.parametrize("smol", [H.FD, H.FV])
def test_stress_force(lattice, smol):
    """Force as the divergence of the stress of Eq. (muf), two-phase (B != 0)."""
    c = H.config(lattice=lattice, smol=smol, shape=SHAPES[lattice], a=-0.04, b=0.04,
                 kappa=0.05, init=1, kT=1e-5, force_form=1)
    _check(c, 20)


@pytest.mark.parametrize("lattice", [H.D2Q9, H.D3Q19])
def test_stress_force_fp32dev(lattice):
    c = H.config(lattice=lattice, smol=H.FV, precision=H.FP32DEV, shape=SHAPES[lattice],
                 a=-0.04, b=0.04, init=1, force_form=1)
    _check(c, 20)


@pytest.mark.parametrize("lattice,smol", [(H.D2Q9, H.FD), (H.D3Q19, H.FV), (H.D3Q15, H.FD)])
def test_stress_force_conserves_momentum_on_gpu(lattice, smol):
    """With B != 0 the total momentum is constant to rounding under the
    stress-divergence force and drifts under -psi grad mu."""
    from paper_1104_0078_amd import lbl
    drift = {}
    for ff in (1, 0):
        c = H.config(lattice=lattice, smol=smol, shape=SHAPES[lattice], a=-0.04, b=0.04,
                     kappa=0.05, init=1, kT=1e-5, force_form=ff)
        with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-2)) as sim:
            t0 = sim.observe(lbl.LBL_OBS_TOTALS)
            sim.step(200)
            t1 = sim.observe(lbl.LBL_OBS_TOTALS)
        scale = t1[6:9].sum()
        drift[ff] = np.abs(t1[1:4] - t0[1:4]).max() / scale
    print("  momentum drift / sum|j|: stress %.2e, psi grad mu %.2e" % (drift[1], drift[0]))
    assert drift[1] < 1e-12
    assert drift[0] > 100 * drift[1]


def test_stress_force_velocity_observable():
    from paper_1104_0078_amd import lbl
    import oracle as O
    c = H.config(lattice=H.D3Q19, smol=H.FD, shape=SHAPES[H.D3Q19], a=-0.04, b=0.04, init=1,
                 force_form=1)
    p = H.oracle_params(c)
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3)) as sim:
        sim.step(5)
        u = sim.observe(lbl.LBL_OBS_U)
    f, psi = H.oracle_run(c, 5)
    assert H.rel_err(u, O.velocity(p, f, O.force(p, psi))) < 1e-11


def test_zero_zc_restores_default_chunks():
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=H.D3Q19, smol=H.FV, shape=(24, 20, 40))
    with lbl.Sim(H.lbl_params(c), lbl.make_init()) as sim:
        zc0 = sim.schedule()["zc"]
        sim.set_schedule(lb_width=64, xcd_swizzle=0, zc=5, overlap=0)
        assert sim.schedule()["zc"] == 5
        sim.set_schedule(lb_width=64, xcd_swizzle=0, zc=0, overlap=0)
        assert sim.schedule()["zc"] == zc0
