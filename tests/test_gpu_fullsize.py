"""Parity at the benchmark's full size: the 256^3 D3Q19 + FV two-phase
workload (flat tanh interfaces plus N(0, 1e-3) noise, a = -0.04, b = 0.04,
kappa = 0.05, M = 0.1, kT = 1e-5, eta = 0.1), in the launch schedules the
benchmark picks between, against the FP64 oracle run on the host over the
whole periodic lattice for two steps.  Compared: 200 000 sampled sites of
every population and of psi, and every site of one z-plane through an
interface.  Conservation is checked on the whole lattice with the FP64
reductions.  Bars as for the small cases: 1e-12 (FP64), 1e-5 (FP32-dev),
relative to the largest magnitude of the oracle field."""
import numpy as np
import pytest

import oracle as O
from tests import harness as H

pytestmark = pytest.mark.gpu

SHAPE = (256, 256, 256)
NSTEPS = 2


@pytest.fixture(scope="module")
def oracle_state():
    c = H.config(lattice=H.D3Q19, smol=H.FV, shape=SHAPE, a=-0.04, b=0.04, kappa=0.05, M=0.1,
                 kT=1e-5, eta=0.1, init=1, psi_std=1e-3)
    print("full-size oracle: %s, %d steps" % (SHAPE, NSTEPS), flush=True)
    f, psi = H.oracle_run(c, NSTEPS)
    return c, f.reshape(19, -1), psi.reshape(-1)


def _sample_sites(N, rng):
    idx = rng.choice(N, size=200000, replace=False)
    plane = SHAPE[2] // 4  # an interface sits at z = L/4
    row = np.arange(SHAPE[0] * SHAPE[1]) + plane * SHAPE[0] * SHAPE[1]
    return np.unique(np.concatenate([idx, row]))


@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
@pytest.mark.parametrize("schedule", [None, dict(lb_width=128, xcd_swizzle=0, zc=64),
                                      dict(lb_width=256, xcd_swizzle=3, zc=16)])
def test_full_size_sampled_parity(oracle_state, precision, schedule):
    import torch
    from paper_1104_0078_amd import lbl
    c0, f_ref, psi_ref = oracle_state
    c = dict(c0, precision=precision)
    print("full-size case: precision %d schedule %s" % (precision, schedule), flush=True)
    N = SHAPE[0] * SHAPE[1] * SHAPE[2]
    sites = torch.from_numpy(_sample_sites(N, np.random.default_rng(7))).cuda()
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3)) as sim:
        if schedule is not None:
            sim.set_schedule(**schedule)
        tot0 = sim.observe(lbl.LBL_OBS_TOTALS)
        sim.step(NSTEPS)
        tot1 = sim.observe(lbl.LBL_OBS_TOTALS)
        pop = torch.empty(19 * N, dtype=torch.float64, device="cuda")
        sim.observe_into(lbl.LBL_OBS_POP, pop)
        f_gpu = pop.view(19, N)[:, sites].cpu().numpy()
        del pop
        psi = torch.empty(N, dtype=torch.float64, device="cuda")
        sim.observe_into(lbl.LBL_OBS_PSI, psi)
        psi_gpu = psi[sites].cpu().numpy()
        del psi
    s = sites.cpu().numpy()
    tol = H.TOL[precision]
    ef = float(np.abs(f_gpu - f_ref[:, s]).max() / np.abs(f_ref).max())
    ep = float(np.abs(psi_gpu - psi_ref[s]).max() / np.abs(psi_ref).max())
    print("  rel err populations %.3e psi %.3e over %d sites" % (ef, ep, s.size), flush=True)
    assert ef <= tol and ep <= tol
    # Mass and total psi: exact conservation up to the FP64 reductions
    # (FP32 storage rounds each update).
    ctol = 1e-13 if precision == H.FP64 else 1e-6
    assert abs(tot1[0] - tot0[0]) <= ctol * abs(tot0[0])
    assert abs(tot1[4] - tot0[4]) <= ctol * tot0[9] + 1e-300


SHAPE_W = (128, 128, 128)
WINDOW = 100


@pytest.fixture(scope="module")
def oracle_window():
    """The same two-phase workload on a 128^3 lattice, 100 oracle steps (the
    acceptance window)."""
    c = H.config(lattice=H.D3Q19, smol=H.FV, shape=SHAPE_W, a=-0.04, b=0.04, kappa=0.05,
                 M=0.1, kT=1e-5, eta=0.1, init=1, psi_std=1e-3)
    print("window oracle: %s, %d steps" % (SHAPE_W, WINDOW), flush=True)
    f, psi = H.oracle_run(c, WINDOW)
    return c, f.reshape(19, -1), psi.reshape(-1)


@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_window_128_sampled_parity(oracle_window, precision):
    """100 steps of the 128^3 two-phase workload: 200 000 sampled sites and
    the interface plane z = L/4 against the oracle, FP64 within 1e-12 and
    FP32-deviation within 1e-5."""

    from paper_1104_0078_amd import lbl
    c0, f_ref, psi_ref = oracle_window
    c = dict(c0, precision=precision)
    print("window case: 128^3 precision %d, %d steps" % (precision, WINDOW), flush=True)
    N = SHAPE_W[0] * SHAPE_W[1] * SHAPE_W[2]
    rng = np.random.default_rng(11)
    idx = rng.choice(N, size=200000, replace=False)
    row = np.arange(SHAPE_W[0] * SHAPE_W[1]) + (SHAPE_W[2] // 4) * SHAPE_W[0] * SHAPE_W[1]
    s = np.unique(np.concatenate([idx, row]))
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3)) as sim:
        sim.step(WINDOW)
        f_gpu = sim.observe(lbl.LBL_OBS_POP).reshape(19, N)[:, s]
        psi_gpu = sim.observe(lbl.LBL_OBS_PSI)[s]
    ef = float(np.abs(f_gpu - f_ref[:, s]).max() / np.abs(f_ref).max())
    ep = float(np.abs(psi_gpu - psi_ref[s]).max() / np.abs(psi_ref).max())
    print("  rel err populations %.3e psi %.3e over %d sites" % (ef, ep, s.size), flush=True)
    tol = H.TOL[precision]
    assert ef <= tol and ep <= tol


@pytest.fixture(scope="module")
def oracle_walls():
    """The same 256^3 two-phase workload between walls sliding at
    (0.02, -0.01, 0) and (-0.015, 0.01, 0), as the bench's walls leg runs it;
    two oracle steps over the whole lattice."""
    c = H.config(lattice=H.D3Q19, smol=H.FV, shape=SHAPE, a=-0.04, b=0.04, kappa=0.05, M=0.1,
                 kT=1e-5, eta=0.1, init=1, psi_std=1e-3, walls=1,
                 u_wall=((0.02, -0.01, 0.0), (-0.015, 0.01, 0.0)))
    print("full-size walls oracle: %s, %d steps" % (SHAPE, NSTEPS), flush=True)
    f, psi = H.oracle_run(c, NSTEPS)
    return c, f.reshape(19, -1), psi.reshape(-1)


@pytest.mark.parametrize("precision", [H.FP64, H.FP32DEV])
def test_full_size_walls_sampled_parity(oracle_walls, precision):
    """256^3 between sliding walls: 200 000 sampled sites plus both wall
    layers and the interface plane against the oracle (1e-12 FP64, 1e-5
    FP32-dev), and conservation of mass and psi."""
    import torch
    from paper_1104_0078_amd import lbl
    c0, f_ref, psi_ref = oracle_walls
    c = dict(c0, precision=precision)
    print("full-size walls case: precision %d" % precision, flush=True)
    N = SHAPE[0] * SHAPE[1] * SHAPE[2]
    plane = SHAPE[0] * SHAPE[1]
    rng = np.random.default_rng(13)
    rows = [np.arange(plane) + z * plane for z in (0, SHAPE[2] // 4, SHAPE[2] - 1)]
    s_np = np.unique(np.concatenate([rng.choice(N, size=200000, replace=False)] + rows))
    sites = torch.from_numpy(s_np).cuda()
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3)) as sim:
        tot0 = sim.observe(lbl.LBL_OBS_TOTALS)
        sim.step(NSTEPS)
        tot1 = sim.observe(lbl.LBL_OBS_TOTALS)
        pop = torch.empty(19 * N, dtype=torch.float64, device="cuda")
        sim.observe_into(lbl.LBL_OBS_POP, pop)
        f_gpu = pop.view(19, N)[:, sites].cpu().numpy()
        del pop
        psi = torch.empty(N, dtype=torch.float64, device="cuda")
        sim.observe_into(lbl.LBL_OBS_PSI, psi)
        psi_gpu = psi[sites].cpu().numpy()
        del psi
    tol = H.TOL[precision]
    ef = float(np.abs(f_gpu - f_ref[:, s_np]).max() / np.abs(f_ref).max())
    ep = float(np.abs(psi_gpu - psi_ref[s_np]).max() / np.abs(psi_ref).max())
    print("  rel err populations %.3e psi %.3e over %d sites" % (ef, ep, s_np.size), flush=True)
    assert ef <= tol and ep <= tol
    ctol = 1e-13 if precision == H.FP64 else 1e-6
    assert abs(tot1[0] - tot0[0]) <= ctol * abs(tot0[0])
    assert abs(tot1[4] - tot0[4]) <= ctol * tot0[9] + 1e-300
