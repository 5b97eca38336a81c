"""Thin ctypes binding of the C ABI in include/lbl.h (liblbl.so, gfx950).

Argument marshalling only: every step of the sweep runs in the HIP library.
The functions ``lbl_create``, ``lbl_step``, ``lbl_observe``, ``lbl_destroy``,
``lbl_strerror``, ``lbl_last_error``, ``lbl_abi_version`` and
``lbl_observable_bytes`` mirror the C entry points.  ``Sim`` is a small
convenience wrapper that takes its device memory from PyTorch's caching
allocator and its stream from ``torch.cuda.current_stream()``.

The library must have been built (``__graft_entry__.build()``); importing this
module without it raises, and there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbl.so")

LBL_OK = 0
LBL_E_INVAL, LBL_E_NOMEM, LBL_E_DEVICE = -1, -2, -3
LBL_E_NONFINITE, LBL_E_BUFSIZE, LBL_E_UNSUPPORTED = -4, -5, -6
LBL_D2Q9, LBL_D3Q15, LBL_D3Q19 = 9, 15, 19
LBL_SMOL_FD, LBL_SMOL_FV = 0, 1
LBL_FP64, LBL_FP32DEV = 0, 1
LBL_FULL, LBL_SMOL_ONLY, LBL_LB_ONLY = 0, 1, 2
LBL_INIT_REST, LBL_INIT_TANH_2IF, LBL_INIT_USER = 0, 1, 2
LBL_FDNOISE_LINK, LBL_FDNOISE_FOURIER = 0, 1
LBL_FORCE_PSI_GRAD_MU, LBL_FORCE_STRESS = 0, 1
LBL_WALLS_PERIODIC, LBL_WALLS_LAST = 0, 1
(LBL_OBS_PSI, LBL_OBS_RHO, LBL_OBS_U, LBL_OBS_POP, LBL_OBS_TOTALS, LBL_OBS_SK_AXES,
 LBL_OBS_UK_AXES, LBL_OBS_STEP, LBL_OBS_NSAMPLES, LBL_OBS_PSIK_AXES, LBL_OBS_SK2_AXES,
 LBL_OBS_UK2_AXES, LBL_OBS_SK_FULL, LBL_OBS_HEIGHTS) = range(14)


class lbl_params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("smol", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("coupling", ctypes.c_int32), ("rk_stages", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("rho", ctypes.c_double), ("eta", ctypes.c_double), ("M", ctypes.c_double),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("kappa", ctypes.c_double),
        ("kT", ctypes.c_double), ("omega_bulk", ctypes.c_double),
        ("omega_ghost", ctypes.c_double), ("u_imposed", ctypes.c_double * 3),
        ("seed", ctypes.c_uint64), ("sample_every", ctypes.c_int32),
        ("fd_noise", ctypes.c_int32), ("force_form", ctypes.c_int32),
        ("sample_full_k", ctypes.c_int32), ("walls", ctypes.c_int32),
        ("reserved", ctypes.c_int32), ("u_wall", (ctypes.c_double * 3) * 2),
    ]


class lbl_init(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("user_on_device", ctypes.c_int32),
        ("psi_std", ctypes.c_double), ("boost_u", ctypes.c_double * 3),
        ("psi0", ctypes.POINTER(ctypes.c_double)), ("f0", ctypes.POINTER(ctypes.c_double)),
        ("step0", ctypes.c_int64),
    ]


class lbl_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class lbl_schedule(ctypes.Structure):
    _fields_ = [("lb_width", ctypes.c_int32), ("xcd_swizzle", ctypes.c_int32),
                ("zc", ctypes.c_int32), ("overlap", ctypes.c_int32)]


class lbl_pool_info(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_uint64), ("used_bytes", ctypes.c_uint64),
                ("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("done", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("ticks", ctypes.c_int64), ("site_updates", ctypes.c_int64)]


LBL_REQ_QUEUED, LBL_REQ_RUNNING, LBL_REQ_DONE, LBL_REQ_FAILED = 0, 1, 2, 3
LBL_KEEP_PSI = 1
LBL_RES_SK_AXES, LBL_RES_TOTALS, LBL_RES_TIMES, LBL_RES_PSI = 0, 1, 2, 3

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class lbl_env(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32), ("reserved", ctypes.c_int32), ("stream", ctypes.c_void_p),
        ("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p),
    ]


_lib = None


def library():
    """Load liblbl.so; raises if it has not been built.

    torch is imported first: it brings its own HIP runtime, and the library's
    HIP dependency must resolve to that same, already loaded runtime, so that
    device memory and streams from torch and the library's kernels live in one
    runtime instance (loading the library first would start a second one)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (see above: load torch's HIP runtime first)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "liblbl.so is not built (run __graft_entry__.build()); the sweep has no "
                "fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.lbl_create.argtypes = [P(lbl_params), P(lbl_init), P(lbl_env), P(ctypes.c_void_p)]
        L.lbl_create.restype = ctypes.c_int
        L.lbl_step.argtypes = [ctypes.c_void_p, ctypes.c_int64]
        L.lbl_step.restype = ctypes.c_int
        L.lbl_observe.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_int]
        L.lbl_observe.restype = ctypes.c_int
        L.lbl_observable_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.lbl_observable_bytes.restype = ctypes.c_size_t
        L.lbl_destroy.argtypes = [ctypes.c_void_p]
        L.lbl_destroy.restype = ctypes.c_int
        L.lbl_strerror.argtypes = [ctypes.c_int]
        L.lbl_strerror.restype = ctypes.c_char_p
        L.lbl_last_error.argtypes = [ctypes.c_void_p]
        L.lbl_last_error.restype = ctypes.c_char_p
        L.lbl_timing_enable.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.lbl_timing_enable.restype = ctypes.c_int
        L.lbl_timing_read.argtypes = [ctypes.c_void_p, ctypes.POINTER(lbl_kernel_time),
                                      ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
        L.lbl_timing_read.restype = ctypes.c_int
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.lbl_diag_normals.argtypes = [i32, i32, ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_uint32, i64, i32,
                                       P(ctypes.c_double)]
        L.lbl_diag_normals.restype = ctypes.c_int
        L.lbl_set_schedule.argtypes = [vp, P(lbl_schedule)]
        L.lbl_set_schedule.restype = ctypes.c_int
        L.lbl_get_schedule.argtypes = [vp, P(lbl_schedule)]
        L.lbl_get_schedule.restype = ctypes.c_int
        L.lbl_sim_bytes.argtypes = [P(lbl_params)]
        L.lbl_sim_bytes.restype = ctypes.c_uint64
        L.lbl_pool_create.argtypes = [ctypes.c_uint64, P(lbl_env), P(vp)]
        L.lbl_pool_submit.argtypes = [vp, P(lbl_params), P(lbl_init), i64, i32, P(i64)]
        L.lbl_pool_run.argtypes = [vp, i64, P(i64)]
        L.lbl_pool_poll.argtypes = [vp, i64, P(i32), P(i64)]
        L.lbl_pool_result.argtypes = [vp, i64, i32, vp, ctypes.c_size_t]
        L.lbl_pool_result_bytes.argtypes = [vp, i64, i32]
        L.lbl_pool_result_bytes.restype = ctypes.c_size_t
        L.lbl_pool_release.argtypes = [vp, i64]
        L.lbl_pool_stats.argtypes = [vp, P(lbl_pool_info)]
        L.lbl_pool_set_schedule.argtypes = [vp, P(lbl_schedule)]
        L.lbl_pool_get_schedule.argtypes = [vp, P(lbl_schedule)]
        L.lbl_pool_destroy.argtypes = [vp]
        L.lbl_pool_last_error.argtypes = [vp]
        L.lbl_pool_last_error.restype = ctypes.c_char_p
        for n in ("lbl_pool_create", "lbl_pool_submit", "lbl_pool_run", "lbl_pool_poll",
                  "lbl_pool_result", "lbl_pool_release", "lbl_pool_stats",
                  "lbl_pool_set_schedule", "lbl_pool_get_schedule", "lbl_pool_destroy"):
            getattr(L, n).restype = ctypes.c_int
        L.lbl_step_static.argtypes = [P(lbl_params), vp, i64, i64, vp, vp]
        L.lbl_step_static.restype = ctypes.c_int
        L.lbl_abi_version.argtypes = []
        L.lbl_abi_version.restype = ctypes.c_int
        _lib = L
    return _lib


class LblError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (lbl_strerror(code), code, msg))
        self.code = code


def lbl_abi_version():
    return library().lbl_abi_version()


def lbl_strerror(code):
    return library().lbl_strerror(code).decode()


def lbl_last_error(sim=None):
    return library().lbl_last_error(sim).decode()


def lbl_create(params, init, env):
    out = ctypes.c_void_p()
    rc = library().lbl_create(ctypes.byref(params), ctypes.byref(init), ctypes.byref(env),
                              ctypes.byref(out))
    return rc, out


def lbl_step(sim, nsteps):
    return library().lbl_step(sim, nsteps)


def lbl_observe(sim, what, dst_ptr, nbytes, dst_is_device):
    return library().lbl_observe(sim, what, dst_ptr, nbytes, dst_is_device)


def lbl_step_static(params, stream, step0, nsteps, pop_ptr, psi_ptr):
    """Advance the device state (pop, psi) by nsteps steps without allocating
    (workspace of LBL_STATIC_SCRATCH_BYTES per device).  pop_ptr and psi_ptr
    are device addresses; stream a hipStream_t handle (0: null stream)."""
    return library().lbl_step_static(ctypes.byref(params), ctypes.c_void_p(stream),
                                     int(step0), int(nsteps), ctypes.c_void_p(pop_ptr),
                                     ctypes.c_void_p(psi_ptr))


LBL_STATIC_SCRATCH_BYTES = 64 << 20


def lbl_observable_bytes(sim, what):
    return library().lbl_observable_bytes(sim, what)


def lbl_destroy(sim):
    return library().lbl_destroy(sim)


def lbl_timing_enable(sim, enable):
    return library().lbl_timing_enable(sim, int(enable))


def lbl_timing_read(sim, max_entries=32):
    buf = (lbl_kernel_time * max_entries)()
    n = ctypes.c_int()
    rc = library().lbl_timing_read(sim, buf, max_entries, ctypes.byref(n))
    return rc, [(buf[k].name.decode(), int(buf[k].launches), float(buf[k].total_ms))
                for k in range(min(n.value, max_entries))]


def make_params(lattice=LBL_D2Q9, smol=LBL_SMOL_FD, precision=LBL_FP64, coupling=LBL_FULL,
                rk_stages=2, shape=(64, 64, 1), rho=1.0, eta=0.1, M=0.1, a=0.04, b=0.1,
                kappa=0.05, kT=1e-5, omega_bulk=1.0, omega_ghost=1.0, u_imposed=(0, 0, 0),
                seed=1234, sample_every=0, fd_noise=LBL_FDNOISE_LINK,
                force_form=LBL_FORCE_PSI_GRAD_MU, sample_full_k=0, walls=LBL_WALLS_PERIODIC,
                u_wall=((0, 0, 0), (0, 0, 0))):
    nx, ny, nz = (tuple(shape) + (1, 1, 1))[:3]
    p = lbl_params()
    p.lattice, p.smol, p.precision, p.coupling, p.rk_stages = (lattice, smol, precision,
                                                               coupling, rk_stages)
    p.nx, p.ny, p.nz = nx, ny, nz
    p.rho, p.eta, p.M, p.a, p.b, p.kappa, p.kT = rho, eta, M, a, b, kappa, kT
    p.omega_bulk, p.omega_ghost = omega_bulk, omega_ghost
    for k in range(3):
        p.u_imposed[k] = float(u_imposed[k])
    p.seed = seed
    p.sample_every = sample_every
    p.fd_noise = fd_noise
    p.force_form = force_form
    p.sample_full_k = sample_full_k
    p.walls = walls
    for w in range(2):
        for k in range(3):
            p.u_wall[w][k] = float(u_wall[w][k])
    return p


def diag_normals(precision, seed, step, tag, site0, n_sites, n_slots, device=0):
    """Normals the sweep draws for sites site0 .. site0+n_sites-1, slots
    0 .. n_slots-1 (array [site][slot], FP64)."""
    out = np.zeros((int(n_sites), int(n_slots)))
    rc = library().lbl_diag_normals(int(device), int(precision), int(seed), int(step), int(tag),
                                    int(site0), int(n_sites), int(n_slots),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if rc != LBL_OK:
        raise LblError(rc, "lbl_diag_normals")
    return out


def make_init(kind=LBL_INIT_REST, psi_std=1e-3, boost=(0, 0, 0), f0=None, psi0=None, step0=0):
    """f0 (q, N) and psi0 (N,) float64 numpy arrays for LBL_INIT_USER; step0
    is the step counter of the initial state (resume)."""
    ini = lbl_init()
    ini.kind = kind
    ini.step0 = int(step0)
    ini.user_on_device = 0
    ini.psi_std = psi_std
    for k in range(3):
        ini.boost_u[k] = float(boost[k]) if k < len(boost) else 0.0
    keep = []
    if kind == LBL_INIT_USER:
        f0 = np.ascontiguousarray(f0, dtype=np.float64)
        psi0 = np.ascontiguousarray(psi0, dtype=np.float64)
        keep = [f0, psi0]
        ini.f0 = f0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        ini.psi0 = psi0.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    ini._keep = keep
    return ini


class TorchMemory:
    """lbl_env callbacks backed by torch's caching allocator on one device."""

    def __init__(self, device=0, stream=None):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)

        def _alloc(ctx, nbytes, stream):
            try:
                return self.torch.cuda.caching_allocator_alloc(int(nbytes), self.device,
                                                               self.stream)
            except RuntimeError:
                return None

        def _free(ctx, ptr, stream):
            self.torch.cuda.caching_allocator_delete(ptr)

        self._alloc = ALLOC_FN(_alloc)
        self._free = FREE_FN(_free)

    def env(self):
        e = lbl_env()
        e.device = self.device
        e.stream = self.stream.cuda_stream
        e.alloc = self._alloc
        e.free = self._free
        e.ctx = None
        return e


class Sim:
    """One simulation handle on one GPU (device memory from torch)."""

    def __init__(self, params, init=None, device=0, stream=None, memory=None):
        self.params = params
        self.init = init if init is not None else make_init()
        self.memory = memory if memory is not None else TorchMemory(device, stream)
        self.env = self.memory.env()
        rc, h = lbl_create(params, self.init, self.env)
        if rc != LBL_OK:
            raise LblError(rc, lbl_last_error(None))
        self.handle = h
        self.d = 2 if params.lattice == LBL_D2Q9 else 3
        self.q = params.lattice
        self.N = params.nx * params.ny * params.nz

    def step(self, nsteps=1):
        rc = lbl_step(self.handle, nsteps)
        if rc != LBL_OK:
            raise LblError(rc, lbl_last_error(self.handle))

    def observe(self, what):
        nbytes = lbl_observable_bytes(self.handle, what)
        if what in (LBL_OBS_STEP, LBL_OBS_NSAMPLES):
            out = np.zeros(1, dtype=np.int64)
        else:
            out = np.zeros(nbytes // 8, dtype=np.float64)
        rc = lbl_observe(self.handle, what, out.ctypes.data, nbytes, 0)
        if rc != LBL_OK:
            raise LblError(rc, lbl_last_error(self.handle))
        if what == LBL_OBS_POP:
            return out.reshape(self.q, self.N)
        if what == LBL_OBS_U:
            return out.reshape(self.d, self.N)
        if what in (LBL_OBS_STEP, LBL_OBS_NSAMPLES):
            return int(out[0])
        L = max(self.params.nx, self.params.ny, self.params.nz)
        if what in (LBL_OBS_SK_AXES, LBL_OBS_SK2_AXES):
            return out.reshape(self.d, L)
        if what in (LBL_OBS_UK_AXES, LBL_OBS_UK2_AXES):
            return out.reshape(self.d, self.d, L)
        if what == LBL_OBS_PSIK_AXES:
            o = out.reshape(self.d, L, 2)
            return o[..., 0] + 1j * o[..., 1]
        if what == LBL_OBS_SK_FULL:
            p = self.params
            return out.reshape(p.nz, p.ny, p.nx // 2 + 1)
        if what == LBL_OBS_HEIGHTS:
            p = self.params
            return out.reshape(2, p.ny, p.nx) if self.d == 3 else out.reshape(2, p.nx)
        return out

    def observe_into(self, what, tensor):
        """Write an observable into a torch CUDA tensor (float64/int64) on the device."""
        nbytes = lbl_observable_bytes(self.handle, what)
        if tensor.numel() * tensor.element_size() < nbytes:
            raise ValueError("tensor too small")
        rc = lbl_observe(self.handle, what, tensor.data_ptr(), tensor.numel() *
                         tensor.element_size(), 1)
        if rc != LBL_OK:
            raise LblError(rc, lbl_last_error(self.handle))
        return tensor

    def timing(self, enable=True):
        rc = lbl_timing_enable(self.handle, enable)
        if rc != LBL_OK:
            raise LblError(rc, lbl_last_error(self.handle))

    def kernel_times(self):
        """[(kernel name, launches, total ms)] since timing was enabled."""
        rc, rows = lbl_timing_read(self.handle)
        if rc != LBL_OK:
            raise LblError(rc, lbl_last_error(self.handle))
        return rows

    def set_schedule(self, lb_width=None, xcd_swizzle=None, zc=0, overlap=None):
        """Launch schedule (speed only): LB block width along x (32..256),
        XCD-contiguous block order (bit 0: LB kernels, bit 1: SMOL tiles),
        planes per SMOL tile (0 keeps), first stage on a second stream."""
        cur = self.schedule()
        sch = lbl_schedule(int(lb_width if lb_width is not None else cur["lb_width"]),
                           int(xcd_swizzle if xcd_swizzle is not None else cur["xcd_swizzle"]),
                           int(zc), int(overlap if overlap is not None else cur["overlap"]))
        rc = library().lbl_set_schedule(self.handle, ctypes.byref(sch))
        if rc != LBL_OK:
            raise LblError(rc, lbl_last_error(self.handle))

    def schedule(self):
        sch = lbl_schedule()
        rc = library().lbl_get_schedule(self.handle, ctypes.byref(sch))
        if rc != LBL_OK:
            raise LblError(rc, lbl_last_error(self.handle))
        return {"lb_width": sch.lb_width, "xcd_swizzle": sch.xcd_swizzle, "zc": sch.zc,
                "overlap": sch.overlap}

    def close(self):
        if getattr(self, "handle", None):
            lbl_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def lbl_sim_bytes(params):
    return int(library().lbl_sim_bytes(ctypes.byref(params)))


class Pool:
    """Many independent simulations batched on one GPU (lbl_pool_* entry points)."""

    def __init__(self, budget_bytes, device=0, stream=None, memory=None):
        self.memory = memory if memory is not None else TorchMemory(device, stream)
        self.env = self.memory.env()
        h = ctypes.c_void_p()
        rc = library().lbl_pool_create(int(budget_bytes), ctypes.byref(self.env), ctypes.byref(h))
        if rc != LBL_OK:
            raise LblError(rc, lbl_last_error(None))
        self.handle = h
        self.params = {}

    def _check(self, rc):
        if rc != LBL_OK:
            raise LblError(rc, library().lbl_pool_last_error(self.handle).decode())

    def submit(self, params, init=None, nsteps=0, keep_psi=False):
        init = init if init is not None else make_init()
        rid = ctypes.c_int64()
        rc = library().lbl_pool_submit(self.handle, ctypes.byref(params), ctypes.byref(init),
                                       int(nsteps), LBL_KEEP_PSI if keep_psi else 0,
                                       ctypes.byref(rid))
        self._check(rc)
        self.params[rid.value] = params
        return rid.value

    def run(self, max_steps):
        pending = ctypes.c_int64()
        self._check(library().lbl_pool_run(self.handle, int(max_steps), ctypes.byref(pending)))
        return pending.value

    def poll(self, rid):
        st, done = ctypes.c_int32(), ctypes.c_int64()
        self._check(library().lbl_pool_poll(self.handle, rid, ctypes.byref(st),
                                            ctypes.byref(done)))
        return st.value, done.value

    def result(self, rid, what):
        n = library().lbl_pool_result_bytes(self.handle, rid, what)
        out = np.zeros(max(1, n // 8))
        self._check(library().lbl_pool_result(self.handle, rid, what, out.ctypes.data, n))
        p = self.params.get(rid)
        if what == LBL_RES_SK_AXES and p is not None:
            d = 2 if p.lattice == LBL_D2Q9 else 3
            return out.reshape(d, max(p.nx, p.ny, p.nz))
        return out

    def release(self, rid):
        self._check(library().lbl_pool_release(self.handle, rid))
        self.params.pop(rid, None)

    def stats(self):
        info = lbl_pool_info()
        self._check(library().lbl_pool_stats(self.handle, ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in lbl_pool_info._fields_}

    def set_schedule(self, lb_width=None, xcd_swizzle=None, zc=None):
        """Work-table schedule of the batched launches (speed only)."""
        cur = self.schedule()
        sch = lbl_schedule(int(lb_width if lb_width is not None else cur["lb_width"]),
                           int(bool(xcd_swizzle if xcd_swizzle is not None
                                    else cur["xcd_swizzle"])),
                           int(zc if zc is not None else cur["zc"]), 0)
        self._check(library().lbl_pool_set_schedule(self.handle, ctypes.byref(sch)))

    def schedule(self):
        sch = lbl_schedule()
        self._check(library().lbl_pool_get_schedule(self.handle, ctypes.byref(sch)))
        return {"lb_width": sch.lb_width, "xcd_swizzle": sch.xcd_swizzle, "zc": sch.zc}

    def close(self):
        if getattr(self, "handle", None):
            library().lbl_pool_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
