"""Test helpers: one configuration, expressed for both the oracle and the HIP
library, plus the comparison measures used by the parity tests.  No method
arithmetic lives here."""
import numpy as np

import oracle as O

D2Q9, D3Q15, D3Q19 = 9, 15, 19
FD, FV = 0, 1
FP64, FP32DEV = 0, 1
FULL, SMOL_ONLY, LB_ONLY = 0, 1, 2

# Tolerances (relative to the largest magnitude of the reference field).
TOL = {FP64: 1e-12, FP32DEV: 1e-5}


def config(lattice=D2Q9, smol=FD, precision=FP64, coupling=FULL, rk=2, shape=(70, 45, 1),
           rho=1.0, eta=0.1, M=0.1, a=0.04, b=0.1, kappa=0.05, kT=1e-5, omega_bulk=1.0,
           omega_ghost=1.0, u_imposed=(0.0, 0.0, 0.0), seed=1234, init=0, psi_std=1e-3,
           boost=(0.0, 0.0, 0.0), fd_noise=0, force_form=0, walls=0,
           u_wall=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))):
    return dict(lattice=lattice, smol=smol, precision=precision, coupling=coupling, rk=rk,
                fd_noise=fd_noise, force_form=force_form, walls=walls,
                u_wall=tuple(tuple(w) for w in u_wall),
                shape=tuple(shape), rho=rho, eta=eta, M=M, a=a, b=b, kappa=kappa, kT=kT,
                omega_bulk=omega_bulk, omega_ghost=omega_ghost, u_imposed=tuple(u_imposed),
                seed=seed, init=init, psi_std=psi_std, boost=tuple(boost))


def oracle_params(c):
    return O.make_params(lattice=c["lattice"], smol=c["smol"], coupling=c["coupling"],
                         rk_stages=c["rk"], shape=c["shape"], rho0=c["rho"], eta=c["eta"],
                         M=c["M"], a=c["a"], b=c["b"], kappa=c["kappa"], kT=c["kT"],
                         omega_bulk=c["omega_bulk"], omega_ghost=c["omega_ghost"],
                         u_imposed=c["u_imposed"], seed=c["seed"], fd_noise=c["fd_noise"],
                         force_form=c["force_form"], walls=c.get("walls", 0),
                         u_wall=tuple(c.get("u_wall", ((0,) * 3, (0,) * 3))[0]) +
                         tuple(c.get("u_wall", ((0,) * 3, (0,) * 3))[1]))


def lbl_params(c, sample_every=0):
    from paper_1104_0078_amd import lbl
    return lbl.make_params(lattice=c["lattice"], smol=c["smol"], precision=c["precision"],
                           coupling=c["coupling"], rk_stages=c["rk"], shape=c["shape"],
                           rho=c["rho"], eta=c["eta"], M=c["M"], a=c["a"], b=c["b"],
                           kappa=c["kappa"], kT=c["kT"], omega_bulk=c["omega_bulk"],
                           omega_ghost=c["omega_ghost"], u_imposed=c["u_imposed"],
                           seed=c["seed"], sample_every=sample_every, fd_noise=c["fd_noise"],
                           force_form=c["force_form"], walls=c.get("walls", 0),
                           u_wall=c.get("u_wall", ((0, 0, 0), (0, 0, 0))))


def oracle_run(c, nsteps, f=None, psi=None):
    p = oracle_params(c)
    if f is None:
        f, psi = O.init(p, c["init"], c["psi_std"], c["boost"])
    O.run(p, f, psi, 0, nsteps)
    return f, psi


def rel_err(got, ref):
    scale = np.abs(ref).max()
    return float(np.abs(np.asarray(got) - ref).max() / (scale if scale > 0 else 1.0))
