"""GPU tests of the pool (batched and served simulations).

* A pooled request gives the same final state as the same simulation run
  alone through lbl_create/lbl_step, and as the FP64 oracle.
* Alone vs in a mix: a request's results do not depend on what else is
  resident or when it was admitted (continuous batching).
* Admission by device-memory budget: requests wait while memory is short,
  a request larger than the whole budget is refused, release cancels.
"""
import numpy as np
import pytest

import oracle as O
from tests import harness as H

pytestmark = pytest.mark.gpu


def _run_pool(pool, chunk=7):
    n = 0
    while pool.run(chunk) > 0:
        n += 1
        assert n < 100000
    return n


def _single(c, nsteps):
    from paper_1104_0078_amd import lbl
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=c["init"], psi_std=c["psi_std"])) as sim:
        sim.step(nsteps)
        return sim.observe(lbl.LBL_OBS_PSI), sim.observe(lbl.LBL_OBS_TOTALS)


MIX = [
    (H.config(lattice=H.D2Q9, smol=H.FD, shape=(48, 40, 1), seed=11), 23),
    (H.config(lattice=H.D2Q9, smol=H.FD, shape=(70, 33, 1), seed=12, a=0.07), 40),
    (H.config(lattice=H.D2Q9, smol=H.FD, precision=H.FP32DEV, shape=(64, 64, 1), seed=13), 31),
    (H.config(lattice=H.D3Q19, smol=H.FV, shape=(20, 14, 12), seed=14), 17),
    (H.config(lattice=H.D3Q19, smol=H.FV, shape=(16, 16, 40), seed=15, a=-0.04, b=0.04,
              init=1), 25),
    (H.config(lattice=H.D2Q9, smol=H.FV, coupling=H.SMOL_ONLY, shape=(40, 40, 1), seed=16,
              u_imposed=(0.02, 0.01, 0)), 19),
    (H.config(lattice=H.D3Q15, smol=H.FD, shape=(12, 18, 10), seed=17), 21),
    # ragged SMOL tiles in x and y, LB rows longer than 64 sites
    (H.config(lattice=H.D3Q19, smol=H.FV, shape=(70, 21, 9), seed=18, a=-0.04, b=0.04,
              init=1), 13),
    # Euler and RK4 stages under full coupling (batched stage kernels with
    # rk = 1 and rk = 4, the RK4 accumulator)
    (H.config(lattice=H.D2Q9, smol=H.FD, shape=(40, 36, 1), seed=19, rk=1, a=-0.04, b=0.04,
              init=1), 15),
    (H.config(lattice=H.D3Q19, smol=H.FV, shape=(18, 14, 12), seed=20, rk=4, a=-0.04, b=0.04,
              init=1), 14),
    (H.config(lattice=H.D2Q9, smol=H.FV, precision=H.FP32DEV, shape=(36, 40, 1), seed=22,
              rk=4), 16),
    # walls across the last axis, sliding; batched in groups of their own
    (H.config(lattice=H.D3Q19, smol=H.FV, shape=(20, 14, 12), seed=23, a=-0.04, b=0.04,
              init=1, walls=1, u_wall=((0.02, -0.01, 0), (-0.015, 0.01, 0))), 18),
    (H.config(lattice=H.D2Q9, smol=H.FV, shape=(36, 28, 1), seed=24, walls=1,
              u_wall=((0.02, 0, 0), (-0.01, 0, 0))), 21),
    (H.config(lattice=H.D3Q15, smol=H.FV, precision=H.FP32DEV, shape=(14, 12, 10), seed=25,
              rk=4, walls=1, u_wall=((0.01, 0.01, 0), (0, 0, 0))), 12),
    # FV on 3-D lattices draws the noise in the velocity pass's launch: a
    # request with the noise and no velocity pass (SMOL alone; Euler), and
    # one with the velocity pass and no noise (kT = 0)
    (H.config(lattice=H.D3Q19, smol=H.FV, coupling=H.SMOL_ONLY, shape=(14, 12, 10), seed=26,
              u_imposed=(0.02, 0.01, -0.01)), 15),
    (H.config(lattice=H.D3Q19, smol=H.FV, shape=(16, 12, 10), seed=27, rk=1, a=-0.04, b=0.04,
              init=1), 13),
    (H.config(lattice=H.D3Q15, smol=H.FV, shape=(12, 10, 14), seed=28, kT=0.0, a=-0.04, b=0.04,
              init=1), 11),
]


def test_pool_matches_single_and_oracle():
    from paper_1104_0078_amd import lbl
    with lbl.Pool(1 << 30) as pool:
        ids = []
        for c, n in MIX:
            ids.append(pool.submit(H.lbl_params(c), lbl.make_init(kind=c["init"],
                                                                  psi_std=c["psi_std"]),
                                   n, keep_psi=True))
        _run_pool(pool)
        for (c, n), rid in zip(MIX, ids):
            st, done = pool.poll(rid)
            assert st == lbl.LBL_REQ_DONE and done == n
            psi_pool = pool.result(rid, lbl.LBL_RES_PSI)
            psi_alone, _ = _single(c, n)
            print("pool vs single", c["lattice"], c["shape"], "max |diff|",
                  np.abs(psi_pool - psi_alone).max(), flush=True)
            np.testing.assert_array_equal(psi_pool, psi_alone)
            if c["precision"] == H.FP64:
                _, psi_ref = H.oracle_run(c, n)
                assert H.rel_err(psi_pool, psi_ref) < 1e-12
            tot = pool.result(rid, lbl.LBL_RES_TOTALS)
            tol = 1e-13 if c["precision"] == H.FP64 else 1e-6
            assert abs(tot[10] - tot[0]) <= tol * tot[5]
            assert abs(tot[14] - tot[4]) <= tol * max(tot[9], 1e-300) * 10 + 1e-12
            t = pool.result(rid, lbl.LBL_RES_TIMES)
            assert t[0] <= t[1] <= t[2]


def test_alone_vs_mix_continuous_batching():
    from paper_1104_0078_amd import lbl
    probe_c, probe_n = MIX[3]
    with lbl.Pool(1 << 30) as pool:
        rid = pool.submit(H.lbl_params(probe_c), lbl.make_init(psi_std=1e-3), probe_n,
                          keep_psi=True)
        _run_pool(pool, chunk=5)
        alone = pool.result(rid, lbl.LBL_RES_PSI)
        alone_sk = pool.result(rid, lbl.LBL_RES_SK_AXES)
    with lbl.Pool(1 << 30) as pool:
        others = [pool.submit(H.lbl_params(c), lbl.make_init(kind=c["init"], psi_std=1e-3), n)
                  for c, n in MIX[:3]]
        pool.run(5)  # the probe arrives while others are running
        rid = pool.submit(H.lbl_params(probe_c), lbl.make_init(psi_std=1e-3), probe_n,
                          keep_psi=True)
        pool.run(3)
        late = [pool.submit(H.lbl_params(c), lbl.make_init(kind=c["init"], psi_std=1e-3), n)
                for c, n in MIX[4:]]
        _run_pool(pool, chunk=4)
        mixed = pool.result(rid, lbl.LBL_RES_PSI)
        mixed_sk = pool.result(rid, lbl.LBL_RES_SK_AXES)
        for r in others + late:
            assert pool.poll(r)[0] == lbl.LBL_REQ_DONE
    np.testing.assert_array_equal(mixed, alone)
    np.testing.assert_array_equal(mixed_sk, alone_sk)


def test_budget_admission_and_release():
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=H.D2Q9, smol=H.FD, shape=(64, 64, 1))
    p = H.lbl_params(c)
    one = lbl.lbl_sim_bytes(p)
    with lbl.Pool(int(2.5 * one)) as pool:
        ids = [pool.submit(p, lbl.make_init(), 10) for _ in range(4)]
        big = H.lbl_params(H.config(lattice=H.D2Q9, shape=(256, 256, 1)))
        with pytest.raises(lbl.LblError) as e:
            pool.submit(big, lbl.make_init(), 10)
        assert e.value.code == lbl.LBL_E_NOMEM
        pool.run(4)
        states = [pool.poll(r)[0] for r in ids]
        assert states == [lbl.LBL_REQ_RUNNING] * 2 + [lbl.LBL_REQ_QUEUED] * 2
        assert pool.stats()["used_bytes"] == 2 * one
        pool.release(ids[1])  # cancel a running request: frees its memory
        assert pool.stats()["used_bytes"] == one
        _run_pool(pool, chunk=4)
        assert [pool.poll(r)[0] for r in (ids[0], ids[2], ids[3])] == [lbl.LBL_REQ_DONE] * 3
        assert pool.stats()["used_bytes"] == 0


def test_schedule_does_not_change_results():
    from paper_1104_0078_amd import lbl
    c, n = MIX[4]
    out = []
    for w, swz, zc in ((64, 0, 0), (64, 1, 0), (128, 1, 8), (32, 0, 40), (256, 1, 0)):
        with lbl.Pool(1 << 30) as pool:
            pool.set_schedule(lb_width=w, xcd_swizzle=swz, zc=zc)
            rid = pool.submit(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3), n,
                              keep_psi=True)
            _run_pool(pool, chunk=6)
            out.append(pool.result(rid, lbl.LBL_RES_PSI))
    for o in out[1:]:
        np.testing.assert_array_equal(o, out[0])


def test_nonfinite_request_fails_alone():
    """A request whose state holds a NaN fails on its own; the requests
    batched with it finish with exactly the fields they have alone."""
    from paper_1104_0078_amd import lbl
    import oracle as O
    bad_c = H.config(lattice=H.D2Q9, smol=H.FD, shape=(48, 40, 1), seed=21)
    f0, psi0 = O.init(H.oracle_params(bad_c), 0, 1e-3)
    psi0[77] = np.nan
    good = MIX[:2]
    alone = []
    for c, n in good:
        with lbl.Pool(1 << 30) as pool:
            rid = pool.submit(H.lbl_params(c), lbl.make_init(kind=c["init"], psi_std=1e-3), n,
                              keep_psi=True)
            _run_pool(pool)
            alone.append(pool.result(rid, lbl.LBL_RES_PSI))
    with lbl.Pool(1 << 30) as pool:
        bad = pool.submit(H.lbl_params(bad_c),
                          lbl.make_init(kind=lbl.LBL_INIT_USER, f0=f0, psi0=psi0), 30)
        ids = [pool.submit(H.lbl_params(c), lbl.make_init(kind=c["init"], psi_std=1e-3), n,
                           keep_psi=True) for c, n in good]
        _run_pool(pool)
        assert pool.poll(bad)[0] == lbl.LBL_REQ_FAILED
        for rid, ref in zip(ids, alone):
            assert pool.poll(rid)[0] == lbl.LBL_REQ_DONE
            np.testing.assert_array_equal(pool.result(rid, lbl.LBL_RES_PSI), ref)
        assert pool.stats()["failed"] == 1
