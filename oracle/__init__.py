"""ctypes binding of the plain FP64 CPU oracle (liblbl_oracle.so).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by
the benchmark's CPU-baseline leg, never by the product package.  The oracle
implements one coupled FLBE + SMOL step of arXiv:1104.0078 literally, in FP64,
with plain loops; see lbl_oracle.c for the passage each function follows.

Array conventions (numpy, float64, C order):
  populations f: shape (q, N), canonical velocity order of ``velocities``;
  scalar fields: shape (N,);  vector fields: shape (d, N);
  site index s = x + nx*(y + ny*z).
"""
import ctypes
import os

import numpy as np

from . import build as _build

FD, FV = 0, 1
FULL, SMOL_ONLY, LB_ONLY = 0, 1, 2
D2Q9, D3Q15, D3Q19 = 9, 15, 19
TAG_LB, TAG_SMOL, TAG_INIT = 0, 1, 2
FDNOISE_LINK, FDNOISE_FOURIER = 0, 1
FORCE_PSI_GRAD_MU, FORCE_STRESS = 0, 1


class Params(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("smol", ctypes.c_int32),
        ("coupling", ctypes.c_int32), ("rk_stages", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("fd_noise", ctypes.c_int32),
        ("rho0", ctypes.c_double), ("eta", ctypes.c_double), ("M", ctypes.c_double),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("kappa", ctypes.c_double),
        ("kT", ctypes.c_double), ("omega_bulk", ctypes.c_double),
        ("omega_ghost", ctypes.c_double), ("u_imposed", ctypes.c_double * 3),
        ("seed", ctypes.c_uint64),
        ("force_form", ctypes.c_int32), ("walls", ctypes.c_int32),
        ("u_wall", ctypes.c_double * 6),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        up = ctypes.POINTER(ctypes.c_uint32)
        P = ctypes.POINTER(Params)
        sigs = {
            "orc_q": (ctypes.c_int, [ctypes.c_int]),
            "orc_d": (ctypes.c_int, [ctypes.c_int]),
            "orc_velocities": (None, [ctypes.c_int, ip, dp]),
            "orc_basis": (None, [ctypes.c_int, dp]),
            "orc_nlinks": (ctypes.c_int, [ctypes.c_int]),
            "orc_links": (None, [ctypes.c_int, ip, dp]),
            "orc_philox4x32_10": (None, [up, up, up]),
            "orc_normal": (ctypes.c_double, [ctypes.c_uint64, ctypes.c_uint32,
                                             ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_uint32]),
            "orc_laplacian": (None, [P, dp, dp]),
            "orc_gradient": (None, [P, dp, dp]),
            "orc_divergence": (None, [P, dp, dp]),
            "orc_chemical_potential": (None, [P, dp, dp]),
            "orc_force": (None, [P, dp, dp]),
            "orc_velocity": (None, [P, dp, dp, dp]),
            "orc_fd_noise_divergence": (None, [P, dp, dp]),
            "orc_fd_noise_fourier": (None, [P, dp, dp]),
            "orc_stress": (None, [P, dp, dp]),
            "orc_smol_noise": (None, [P, ctypes.c_uint32, dp]),
            "orc_collide": (None, [P, dp, dp, dp, dp]),
            "orc_smol_rhs": (None, [P, dp, dp, dp, dp]),
            "orc_init": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_double, dp, dp, dp]),
            "orc_step": (ctypes.c_int, [P, dp, dp, ctypes.c_uint32]),
            "orc_run": (ctypes.c_int, [P, dp, dp, ctypes.c_uint32, ctypes.c_int64]),
            "orc_totals": (None, [P, dp, dp, dp]),
            "orc_axis_spectrum": (None, [P, dp, ctypes.c_int32, dp]),
            "orc_heights": (None, [P, dp, dp]),
            "orc_set_threads": (None, [ctypes.c_int32]),
            "orc_max_threads": (ctypes.c_int32, []),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_params(lattice=D2Q9, smol=FD, coupling=FULL, rk_stages=2, shape=(16, 16, 1),
                rho0=1.0, eta=0.1, M=0.1, a=0.04, b=0.1, kappa=0.05, kT=1e-5,
                omega_bulk=1.0, omega_ghost=1.0, u_imposed=(0.0, 0.0, 0.0), seed=1234,
                fd_noise=FDNOISE_LINK, force_form=FORCE_PSI_GRAD_MU, walls=0,
                u_wall=(0.0, 0.0, 0.0, 0.0, 0.0, 0.0)):
    nx, ny, nz = (tuple(shape) + (1, 1, 1))[:3]
    p = Params()
    p.lattice, p.smol, p.coupling, p.rk_stages = lattice, smol, coupling, rk_stages
    p.fd_noise = fd_noise
    p.force_form = force_form
    p.walls = walls
    for k in range(6):
        p.u_wall[k] = float(u_wall[k])
    p.nx, p.ny, p.nz = nx, ny, nz
    p.rho0, p.eta, p.M, p.a, p.b, p.kappa, p.kT = rho0, eta, M, a, b, kappa, kT
    p.omega_bulk, p.omega_ghost = omega_bulk, omega_ghost
    for k in range(3):
        p.u_imposed[k] = float(u_imposed[k])
    p.seed = seed
    return p


def nsites(p):
    return p.nx * p.ny * p.nz


def q_of(p):
    return lib().orc_q(p.lattice)


def d_of(p):
    return lib().orc_d(p.lattice)


def velocities(lattice):
    q = lib().orc_q(lattice)
    c = np.zeros((q, 3), dtype=np.int32)
    w = np.zeros(q)
    lib().orc_velocities(lattice, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(w))
    return c, w


def basis(lattice):
    q = lib().orc_q(lattice)
    E = np.zeros((q, q))
    lib().orc_basis(lattice, _dp(E))
    return E


def links(lattice):
    n = lib().orc_nlinks(lattice)
    c = np.zeros((n, 3), dtype=np.int32)
    lam = np.zeros(n)
    lib().orc_links(lattice, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _dp(lam))
    return c, lam


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def normal(seed, site, step, tag, slot):
    return lib().orc_normal(seed, site, step, tag, slot)


def _unary(name, p, x, out_shape):
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(out_shape)
    getattr(lib(), name)(ctypes.byref(p), _dp(x), _dp(out))
    return out


def laplacian(p, x):
    return _unary("orc_laplacian", p, x, (nsites(p),))


def gradient(p, x):
    return _unary("orc_gradient", p, x, (d_of(p), nsites(p)))


def divergence(p, v):
    return _unary("orc_divergence", p, v, (nsites(p),))


def chemical_potential(p, psi):
    return _unary("orc_chemical_potential", p, psi, (nsites(p),))


def force(p, psi):
    return _unary("orc_force", p, psi, (d_of(p), nsites(p)))


def stress(p, psi):
    """Order-parameter stress of Eq. (muf), full d x d tensor per site."""
    d = d_of(p)
    return _unary("orc_stress", p, psi, (d, d, nsites(p)))


def velocity(p, f, F):
    f = np.ascontiguousarray(f, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    u = np.zeros((d_of(p), nsites(p)))
    lib().orc_velocity(ctypes.byref(p), _dp(f), _dp(F), _dp(u))
    return u


def fd_noise_divergence(p, zeta):
    return _unary("orc_fd_noise_divergence", p, zeta, (nsites(p),))


def fd_noise_fourier(p, w):
    """FD noise built in Fourier space from the white field w (Sec. V.A)."""
    return _unary("orc_fd_noise_fourier", p, w, (nsites(p),))


def smol_noise(p, step):
    out = np.zeros(nsites(p))
    lib().orc_smol_noise(ctypes.byref(p), step, _dp(out))
    return out


def collide(p, fbar, F, r):
    q, d = q_of(p), d_of(p)
    fbar = np.ascontiguousarray(fbar, dtype=np.float64)
    F3 = np.zeros(3)
    F3[:d] = np.asarray(F, dtype=np.float64)[:d]
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.zeros(q)
    lib().orc_collide(ctypes.byref(p), _dp(fbar), _dp(F3), _dp(r), _dp(out))
    return out


def smol_rhs(p, phi, u, noise):
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    noise = np.ascontiguousarray(noise, dtype=np.float64)
    out = np.zeros(nsites(p))
    lib().orc_smol_rhs(ctypes.byref(p), _dp(phi), _dp(u), _dp(noise), _dp(out))
    return out


def init(p, kind=0, psi_std=1e-3, boost=None):
    f = np.zeros((q_of(p), nsites(p)))
    psi = np.zeros(nsites(p))
    b = np.zeros(3)
    if boost is not None:
        b[:len(boost)] = boost
    rc = lib().orc_init(ctypes.byref(p), kind, psi_std, _dp(b), _dp(f), _dp(psi))
    if rc:
        raise ValueError("orc_init rejected the parameters")
    return f, psi


def step(p, f, psi, n):
    rc = lib().orc_step(ctypes.byref(p), _dp(f), _dp(psi), n)
    if rc:
        raise ValueError("orc_step failed")


def run(p, f, psi, step0, nsteps):
    rc = lib().orc_run(ctypes.byref(p), _dp(f), _dp(psi), step0, nsteps)
    if rc:
        raise ValueError("orc_run failed")


def totals(p, f, psi):
    out = np.zeros(10)
    lib().orc_totals(ctypes.byref(p), _dp(np.ascontiguousarray(f)),
                     _dp(np.ascontiguousarray(psi)), _dp(out))
    return out


def axis_spectrum(p, field, lmax=None):
    if lmax is None:
        lmax = max(p.nx, p.ny, p.nz)
    out = np.zeros((3, lmax))
    lib().orc_axis_spectrum(ctypes.byref(p), _dp(np.ascontiguousarray(field, dtype=np.float64)),
                            lmax, _dp(out))
    return out[:d_of(p)]


def heights(p, psi):
    """Interface heights (2, C): the zero crossings of psi along the last axis
    near L/4 and 3L/4 per column (C = nx*ny in 3-D, nx in 2-D)."""
    C = p.nx * p.ny if d_of(p) == 3 else p.nx
    out = np.zeros((2, C))
    lib().orc_heights(ctypes.byref(p), _dp(np.ascontiguousarray(psi, dtype=np.float64)),
                      _dp(out))
    return out


def set_threads(n):
    """OpenMP threads of the oracle's site loops."""
    lib().orc_set_threads(int(n))


def max_threads():
    return int(lib().orc_max_threads())
