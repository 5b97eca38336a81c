"""Error paths of the C ABI on the GPU, forced from the host.  Device
allocation failures are injected through the lbl_env allocator, at every
allocation lbl_create makes and at the staging allocation of lbl_observe: each
must return LBL_E_NOMEM, hand back every allocation already made, and leave a
live simulation usable.  The argument errors of lbl_step and lbl_observe give
the codes the header documents."""

import numpy as np
import pytest

from tests import harness as H

pytestmark = pytest.mark.gpu


class CountingMemory:
    """lbl_env callbacks over torch's caching allocator that count the
    allocations, keep the live ones, and return NULL for the allocation with
    index `fail_at` (counted from 0 over the object's life)."""

    def __init__(self, fail_at=None, device=0):
        import torch
        from paper_1104_0078_amd import lbl
        self.lbl = lbl
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        self.fail_at = fail_at
        self.calls = 0
        self.live = {}
        self.bad_frees = []

        def _alloc(ctx, nbytes, stream):
            k = self.calls
            self.calls += 1
            if self.fail_at is not None and k == self.fail_at:
                return None
            ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            self.live[ptr] = int(nbytes)
            return ptr

        def _free(ctx, ptr, stream):
            if ptr not in self.live:
                self.bad_frees.append(ptr)
                return
            del self.live[ptr]
            torch.cuda.caching_allocator_delete(ptr)

        self._alloc = lbl.ALLOC_FN(_alloc)
        self._free = lbl.FREE_FN(_free)

    def env(self):
        e = self.lbl.lbl_env()
        e.device = self.device
        e.stream = self.stream.cuda_stream
        e.alloc = self._alloc
        e.free = self._free
        e.ctx = None
        return e


CASES = [
    dict(lattice=H.D2Q9, smol=H.FD, shape=(37, 21, 1), init=0),
    dict(lattice=H.D3Q19, smol=H.FV, shape=(13, 11, 9), init=1, a=-0.04, b=0.04),
]


def _user_init(c):
    """A USER initial state, which makes lbl_create stage it through one more
    device allocation."""
    from paper_1104_0078_amd import lbl
    import oracle as O
    f0, psi0 = O.init(H.oracle_params(c), 0, 1e-3)
    return lbl.make_init(kind=lbl.LBL_INIT_USER, f0=f0, psi0=psi0)


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("user", [False, True])
def test_create_allocation_failures(case, user):
    from paper_1104_0078_amd import lbl
    c = H.config(**CASES[case])
    params = H.lbl_params(c, sample_every=1)
    ini = _user_init(c) if user else lbl.make_init(kind=c["init"], psi_std=1e-3)
    print("allocation failures of create:", c["lattice"], c["shape"], "user", user, flush=True)
    probe = CountingMemory()
    with lbl.Sim(params, ini, memory=probe) as sim:
        sim.step(3)
        ref = sim.observe(lbl.LBL_OBS_PSI)
    n_create = probe.calls - 1  # the last allocation staged the observation
    assert n_create >= 17
    assert not probe.live and not probe.bad_frees
    for k in range(n_create):
        mem = CountingMemory(fail_at=k)
        with pytest.raises(lbl.LblError) as e:
            lbl.Sim(params, ini, memory=mem)
        assert e.value.code == lbl.LBL_E_NOMEM, k
        assert mem.calls > k, k
        assert not mem.live and not mem.bad_frees, k
    # A creation after all the failures runs the same trajectory.
    mem = CountingMemory()
    with lbl.Sim(params, ini, memory=mem) as sim:
        sim.step(3)
        np.testing.assert_array_equal(sim.observe(lbl.LBL_OBS_PSI), ref)
    assert not mem.live and not mem.bad_frees


def test_observe_staging_failure_leaves_the_simulation_usable():
    from paper_1104_0078_amd import lbl
    c = H.config(**CASES[1])
    mem = CountingMemory()
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3), memory=mem) as sim:
        sim.step(2)
        n_live = len(mem.live)
        mem.fail_at = mem.calls
        with pytest.raises(lbl.LblError) as e:
            sim.observe(lbl.LBL_OBS_PSI)
        assert e.value.code == lbl.LBL_E_NOMEM
        assert len(mem.live) == n_live
        psi = sim.observe(lbl.LBL_OBS_PSI)
        sim.step(1)
        psi3 = sim.observe(lbl.LBL_OBS_PSI)
        assert sim.observe(lbl.LBL_OBS_STEP) == 3
    assert not mem.live and not mem.bad_frees
    # the failed observation changed nothing
    with lbl.Sim(H.lbl_params(c), lbl.make_init(kind=1, psi_std=1e-3)) as sim:
        sim.step(2)
        np.testing.assert_array_equal(sim.observe(lbl.LBL_OBS_PSI), psi)
        sim.step(1)
        np.testing.assert_array_equal(sim.observe(lbl.LBL_OBS_PSI), psi3)


def test_argument_errors():
    from paper_1104_0078_amd import lbl
    c = H.config(**CASES[0])
    with lbl.Sim(H.lbl_params(c), lbl.make_init()) as sim:
        h = sim.handle
        assert lbl.lbl_step(h, -1) == lbl.LBL_E_INVAL
        assert lbl.lbl_step(h, 0) == lbl.LBL_OK
        n = lbl.lbl_observable_bytes(h, lbl.LBL_OBS_PSI)
        assert n == 8 * 37 * 21
        buf = np.zeros(n // 8 + 1)
        ptr = buf.ctypes.data
        assert lbl.lbl_observe(h, lbl.LBL_OBS_PSI, ptr, n - 1, 0) == lbl.LBL_E_BUFSIZE
        assert lbl.lbl_observe(h, 999, ptr, n, 0) == lbl.LBL_E_INVAL
        assert lbl.lbl_observable_bytes(h, 999) == 0
        assert lbl.lbl_observe(h, lbl.LBL_OBS_PSI, None, n, 0) == lbl.LBL_E_INVAL
        # the whole-zone spectrum exists only when it is sampled
        assert lbl.lbl_observable_bytes(h, lbl.LBL_OBS_SK_FULL) == 0
        assert lbl.lbl_observe(h, lbl.LBL_OBS_SK_FULL, ptr, n, 0) == lbl.LBL_E_INVAL
        # none of these touched the state
        assert lbl.lbl_observe(h, lbl.LBL_OBS_PSI, ptr, n, 0) == lbl.LBL_OK
        assert sim.observe(lbl.LBL_OBS_STEP) == 0
        assert np.all(np.isfinite(buf[:-1])) and buf[-1] == 0.0
    cs = H.config(**dict(CASES[0], coupling=H.SMOL_ONLY))
    with lbl.Sim(H.lbl_params(cs), lbl.make_init()) as sim:
        n = lbl.lbl_observable_bytes(sim.handle, lbl.LBL_OBS_U)
        buf = np.zeros(n // 8)
        rc = lbl.lbl_observe(sim.handle, lbl.LBL_OBS_U, buf.ctypes.data, n, 0)
        assert rc == lbl.LBL_E_UNSUPPORTED
        assert "not available" in lbl.lbl_last_error(sim.handle)
        sim.step(1)
        assert sim.observe(lbl.LBL_OBS_STEP) == 1


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("options", [{}, {"force_form": 1}, {"sample_full_k": 1}])
def test_sim_bytes_match_the_allocations(case, options):
    """The pool admits requests by lbl_sim_bytes: it must equal what
    lbl_create takes through the allocator (zero-sized buffers are taken as 8
    bytes; hipFFT's own work areas are outside the callback)."""
    from paper_1104_0078_amd import lbl
    c = H.config(**CASES[case])
    params = H.lbl_params(c)
    for k, v in options.items():
        setattr(params, k, v)
    mem = CountingMemory()
    with lbl.Sim(params, lbl.make_init(kind=c["init"], psi_std=1e-3), memory=mem):
        taken = sum(mem.live.values())
        n = len(mem.live)
    want = lbl.lbl_sim_bytes(params)
    assert want <= taken <= want + 8 * n


@pytest.mark.parametrize("lattice,shape", [(H.D2Q9, (37, 21, 1)), (H.D3Q19, (13, 11, 9))])
def test_sim_bytes_match_the_allocations_with_walls(lattice, shape):
    """The same with walls (the wall rules live in the kernels; no buffer is
    added)."""
    from paper_1104_0078_amd import lbl
    c = H.config(lattice=lattice, smol=H.FV, shape=shape, walls=1,
                 u_wall=((0.01, 0, 0), (-0.01, 0, 0)))
    params = H.lbl_params(c)
    mem = CountingMemory()
    with lbl.Sim(params, lbl.make_init(psi_std=1e-3), memory=mem) as sim:
        taken = sum(mem.live.values())
        n = len(mem.live)
        sim.step(2)
    want = lbl.lbl_sim_bytes(params)
    assert want <= taken <= want + 8 * n
