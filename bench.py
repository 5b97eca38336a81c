"""Benchmark of the coupled FLBE + SMOL sweep on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                [--no-cpu-baseline] [--no-fp32] [--no-batched] [--no-served]
                [--serve-rate R] [--serve-seconds T] [--no-tune] [--tune-single]
                [--schedule W,S,Z]

Prints ONE JSON line.  A "step" is one full coupled time step (LB collide and
stream with noise, chemical potential, force, SMOL Runge-Kutta with noise) over
the whole lattice, with the state already resident in HBM.  value = lattice
sites x steps / wall time of the timed region (MLUPS, million lattice-site
updates per second) of the plain single-simulation FP64 run.  The kernel
roofline figure is measured live with HIP events on the library's stream
during the same timed region.

Beside it the line carries the FP32-deviation run of the same lattice, the
batched ensemble (96 uneven D2Q9 replicas in one pool, FP32 and FP64) and the
served mix (Poisson arrivals into a pool with an HBM budget; p50/p99
completion latency and aggregate MLUPS).
"""
import argparse
import hashlib
import re
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
METRIC = "coupled FLBE+SMOL MLUPS and % HBM peak, plain FP64 vs batched/served FP32; p50/p99"

# Workloads: synthetic inputs with the structure of the paper's runs (periodic
# lattices, one-phase random or two-phase flat-interface initial states).
WORKLOADS = {
    # Two flat tanh interfaces on 256^3, D3Q19 + finite-volume SMOL, FP64.
    "d3q19_fv_fp64_256_two_phase": dict(lattice=19, smol=1, precision=0, shape=(256, 256, 256),
                                        a=-0.04, b=0.04, kappa=0.05, M=0.1, kT=1e-5, eta=0.1,
                                        init=1, psi_std=1e-3),
    "d3q19_fv_fp32dev_256_two_phase": dict(lattice=19, smol=1, precision=1,
                                           shape=(256, 256, 256), a=-0.04, b=0.04, kappa=0.05,
                                           M=0.1, kT=1e-5, eta=0.1, init=1, psi_std=1e-3),
    # One-phase 128^3, D3Q19 + finite-volume SMOL, FP64.
    "d3q19_fv_fp64_128": dict(lattice=19, smol=1, precision=0, shape=(128, 128, 128), a=0.04,
                              b=0.1, kappa=0.05, M=0.1, kT=1e-5, eta=0.1, init=0, psi_std=1e-3),
    # One-phase 64^2, D2Q9 + finite-difference SMOL, FP64.
    "d2q9_fd_fp64_64": dict(lattice=9, smol=0, precision=0, shape=(64, 64, 1), a=0.04, b=0.1,
                            kappa=0.05, M=0.1, kT=1e-5, eta=0.1, init=0, psi_std=1e-3),
    # One-phase 4096^2, D2Q9 + finite-difference SMOL (HBM-resident 2-D case).
    "d2q9_fd_fp64_4096": dict(lattice=9, smol=0, precision=0, shape=(4096, 4096, 1), a=0.04,
                              b=0.1, kappa=0.05, M=0.1, kT=1e-5, eta=0.1, init=0, psi_std=1e-3),
}
DEFAULT_WORKLOAD = "d3q19_fv_fp64_256_two_phase"


def alg_bytes_per_site(w):
    """Algorithmic HBM bytes of one coupled step per site: the state is read
    once and written once, 2 Q b + 2 b (b = bytes per stored value)."""
    b = 8 if w["precision"] == 0 else 4
    return 2 * w["lattice"] * b + 2 * b


def noise_in_velocity_pass(w, schedule):
    """True when the step draws the SMOL noise inside the velocity pass
    (schedule overlap 3, the default; the noise built in Fourier space is
    drawn apart; the workloads here run full coupling with two stages and
    kT > 0)."""
    return (schedule is not None and schedule.get("overlap") == 3
            and not (w["smol"] == 0 and w.get("fd_noise", 0) == 1))


def kernel_alg_bytes_per_site(name, w, rk=2, schedule=None):
    """Algorithmic bytes per site of one launch of each kernel: every field
    the kernel needs read once and every field it produces written once (no
    halo re-reads); b bytes per stored value, d dimensions.
      k_lb:    pull the Q populations, read psi and mu (force), write the Q
               post-collision populations and u^n:          (2Q + 2 + d) b;
      k_uend:  pull the Q streamed populations, read psi and mu, write the
               stage velocity at t_{n+1}:                   (Q + 2 + d) b,
               and the SMOL noise where it draws it:        + b;
      k_prep:  read psi, write mu and the SMOL noise:        3 b,
               or mu alone where the velocity pass draws the noise: 2 b;
      k_stage: read the stage input, the velocity (d values) and the noise,
               write the output; the final Heun stage also reads psi^n
               (mean over the two launches of a step):      (3 + d) b + b/2."""
    b = 8 if w["precision"] == 0 else 4
    d = 2 if w["lattice"] == 9 else 3
    q = w["lattice"]
    fused = noise_in_velocity_pass(w, schedule)
    if name.startswith("k_lb"):
        return (2 * q + 2 + d) * b
    if name.startswith("k_uend"):
        return (q + 2 + d + (1 if fused else 0)) * b
    if name.startswith("k_prep"):
        return (2 if fused else 3) * b
    if name.startswith("k_stage"):
        return (3 + d) * b + (b / 2 if rk == 2 else 0)
    return None


def state_bytes_per_site(name, w):
    """The part of the step's algorithmic bytes (the state read once and
    written once, 2 Q b + 2 b per site) that one launch of a kernel moves:
    the populations (2 Q b) for the LB passes that collide and stream them;
    None for the kernels whose HBM traffic is the method's intermediate
    fields (chemical potential, noise, velocities, Runge-Kutta stages)."""
    b = 8 if w["precision"] == 0 else 4
    if name == "k_lb":
        return 2 * w["lattice"] * b
    return None


def step_traffic_per_site(ktimes, workload, steps, N):
    """Measured HBM bytes of one whole step per site: the committed counter
    traffic of every kernel (if taken on the current sources) times its
    launches per step; None when a kernel of the step has no current entry."""
    total = 0.0
    for kname, klaunch, _ in ktimes:
        t = traffic_for(kname, workload)
        if t is None:
            return None
        total += t * klaunch / steps
    return total / N


def source_hash():
    """Hash of the kernel sources with comments and white space removed: the
    committed counter summary stays valid across edits of comments alone and
    is dropped by any change of code."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1104_0078_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, fn), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        text = " ".join(text.split())
        h.update(fn.encode())
        h.update(text.encode())
    return h.hexdigest()[:16]


def traffic_for(kernel, workload):
    """HBM traffic per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rows = json.load(open(path))
    except ValueError:
        return None
    for r in rows:
        if (r.get("kernel") == kernel and r.get("workload") == workload
                and r.get("source_hash") == source_hash()):
            return r.get("bytes_per_launch")
    return None


def cpu_baseline(w, workload_name, min_seconds=10.0, max_steps=200, lbl=None):
    """The FP64 oracle, as it stands, on a bounded sample of the same
    workload: steps of the same lattice until at least `min_seconds` of host
    time have passed (at most `max_steps`), timed on the host cores.  With
    the library given, the GPU then takes the same steps from the same
    initial state in FP64 and in FP32-deviation storage, and the errors of
    its psi and populations against the oracle's are reported."""
    import numpy as np
    import oracle as O

    p = O.make_params(lattice=w["lattice"], smol=w["smol"], shape=w["shape"], a=w["a"],
                      b=w["b"], kappa=w["kappa"], M=w["M"], kT=w["kT"], eta=w["eta"],
                      seed=1234)
    f, psi = O.init(p, w["init"], w["psi_std"])
    N = O.nsites(p)
    nsteps, dt = 0, 0.0
    t0 = time.perf_counter()
    while nsteps < max_steps and dt < min_seconds:
        O.run(p, f, psi, nsteps, 1)
        nsteps += 1
        dt = time.perf_counter() - t0
    cores = O.max_threads()
    out = {"value": N * nsteps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": "%d step(s) of %s (%d sites), FP64 oracle, %.1f s" % (
               nsteps, workload_name, N, dt)}
    if lbl is not None:
        def rel(got, ref):
            return float(np.abs(got - ref).max() / np.abs(ref).max())
        err = {"steps": nsteps, "measure": "max |gpu - oracle| / max |oracle| over all sites",
               "bound": {"fp64": 1e-12, "fp32dev": 1e-5}}
        for name, prec in (("fp64", 0), ("fp32dev", 1)):
            init = lbl.make_init(kind=w["init"], psi_std=w["psi_std"])
            with lbl.Sim(make_sim_params(lbl, w, prec), init, device=0) as sim:
                sim.step(nsteps)
                e_psi = rel(sim.observe(lbl.LBL_OBS_PSI), psi)
                e_pop = rel(sim.observe(lbl.LBL_OBS_POP), f)
            err[name] = {"psi": e_psi, "pop": e_pop}
        out["gpu_error_vs_oracle"] = err
    return out


def cpu_model():
    """The host CPU's model name (lscpu), for the baseline's context."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return None


def _oracle_timed(O, p, w, max_steps, min_seconds):
    """Oracle steps from the workload's initial state until min_seconds have
    passed (at most max_steps); returns (f, psi, steps, seconds)."""
    f, psi = O.init(p, w["init"], w["psi_std"])
    nsteps, dt = 0, 0.0
    t0 = time.perf_counter()
    while nsteps < max_steps and dt < min_seconds:
        O.run(p, f, psi, nsteps, 1)
        nsteps += 1
        dt = time.perf_counter() - t0
    return f, psi, nsteps, dt


def cpu_baseline_plan(lbl, torch):
    """The oracle on the small specified workloads, each at one thread and at
    all host threads: D2Q9 + FD 64^2 for its full 2000 steps, and D3Q19 + FV
    128^3 for a bounded number of steps (its 100-step window would take
    minutes on one core).  Beside each, the GPU's rate on the same steps and
    its error against the oracle's fields (FP64 and FP32-deviation)."""
    import numpy as np
    import oracle as O
    nmax = O.max_threads()
    out = []
    for name, steps1, stepsn, min1, minn in (("d2q9_fd_fp64_64", 2000, 2000, 1e9, 1e9),
                                             ("d3q19_fv_fp64_128", 100, 100, 4.0, 8.0)):
        w = WORKLOADS[name]
        p = O.make_params(lattice=w["lattice"], smol=w["smol"], shape=w["shape"], a=w["a"],
                          b=w["b"], kappa=w["kappa"], M=w["M"], kT=w["kT"], eta=w["eta"],
                          seed=1234)
        N = O.nsites(p)
        row = {"workload": name, "sites": N}
        ref = None
        for threads, steps, mins in ((1, steps1, min1), (nmax, stepsn, minn)):
            O.set_threads(threads)
            f, psi, k, dt = _oracle_timed(O, p, w, steps, mins)
            row["threads_%d" % threads] = {"steps": k, "seconds": round(dt, 2),
                                           "mlups": round(N * k / dt / 1e6, 3)}
            if ref is None or k > ref[2]:
                ref = (f, psi, k)
        O.set_threads(nmax)
        f, psi, k = ref
        gpu = {}
        for pname, prec in (("fp64", 0), ("fp32dev", 1)):
            init = lbl.make_init(kind=w["init"], psi_std=w["psi_std"])
            with lbl.Sim(make_sim_params(lbl, w, prec), init, device=0) as sim:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sim.step(k)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                e_psi = float(np.abs(sim.observe(lbl.LBL_OBS_PSI) - psi).max() /
                              np.abs(psi).max())
                e_pop = float(np.abs(sim.observe(lbl.LBL_OBS_POP) - f).max() / np.abs(f).max())
            gpu[pname] = {"mlups": round(N * k / dt / 1e6, 1), "err_psi": e_psi,
                          "err_pop": e_pop}
        row["gpu_same_steps"] = dict(gpu, steps=k,
                                     measure="max |gpu - oracle| / max |oracle| over all sites")
        out.append(row)
    return out


def make_sim_params(lbl, w, precision=None, seed=1234):
    return lbl.make_params(lattice=w["lattice"], smol=w["smol"],
                           precision=w["precision"] if precision is None else precision,
                           shape=w["shape"], rho=1.0, eta=w["eta"], M=w["M"], a=w["a"],
                           b=w["b"], kappa=w["kappa"], kT=w["kT"], seed=seed,
                           fd_noise=w.get("fd_noise", 0), force_form=w.get("force_form", 0),
                           walls=w.get("walls", 0),
                           u_wall=w.get("u_wall", ((0, 0, 0), (0, 0, 0))))


def run_single(lbl, torch, w, wname, steps, warmup, tune, precision=None, schedule=None):
    """Plain single-simulation run: warm-up, then `steps` timed steps."""
    from paper_1104_0078_amd import autotune
    params = make_sim_params(lbl, w, precision)
    init = lbl.make_init(kind=w["init"], psi_std=w["psi_std"])
    stream = torch.cuda.current_stream()
    N = w["shape"][0] * w["shape"][1] * w["shape"][2]
    with lbl.Sim(params, init, device=0, stream=stream) as sim:
        tuned = None
        if schedule is not None:
            sim.set_schedule(**schedule)
        elif tune:
            tuned = autotune.tune_sim(sim, params)
        sim.step(warmup)
        torch.cuda.synchronize()
        sim.timing(True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        sim.step(steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = ev0.elapsed_time(ev1)
        ktimes = sim.kernel_times()
        sim.timing(False)
        tot = sim.observe(lbl.LBL_OBS_TOTALS)
        schedule = sim.schedule()
    seconds = max(wall, gpu_ms / 1e3)
    return {"N": N, "seconds": seconds, "mlups": N * steps / seconds / 1e6,
            "ms_per_step": seconds * 1e3 / steps, "ktimes": ktimes, "totals": tot,
            "schedule": schedule, "tuned_from_cache": None if tuned is None else
            tuned["from_cache"]}


ENSEMBLE_SIDES = (32, 48, 64, 96, 128, 192, 256)


def ensemble_requests(lbl, precision, nrep=96, seed=1234):
    """96 independent D2Q9 + FD replicas: square sides drawn uniformly from
    ENSEMBLE_SIDES, a_r ~ U[0.01, 0.1], b = 0.1, kappa = 0.05, M = 0.1,
    kT = 1e-5, eta = 0.1, Philox seed 1234 + r, psi0 = N(0, 1e-3)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sides = rng.choice(ENSEMBLE_SIDES, size=nrep)
    avals = rng.uniform(0.01, 0.1, size=nrep)
    out = []
    for r in range(nrep):
        L = int(sides[r])
        p = lbl.make_params(lattice=lbl.LBL_D2Q9, smol=lbl.LBL_SMOL_FD, precision=precision,
                            shape=(L, L, 1), rho=1.0, eta=0.1, M=0.1, a=float(avals[r]), b=0.1,
                            kappa=0.05, kT=1e-5, seed=seed + r)
        out.append((p, L * L))
    return out


def run_ensemble(lbl, torch, precision, nsteps, tune, tick=500):
    """All replicas resident in one pool; each tick of `tick` steps of every
    replica is one captured graph, replayed until all are done."""
    from paper_1104_0078_amd import autotune
    reqs = ensemble_requests(lbl, precision)
    init = lbl.make_init(kind=0, psi_std=1e-3)
    sites = sum(n for _, n in reqs)
    res = {"replicas": len(reqs), "sites": sites, "steps": nsteps}
    if tune:
        # Tune on a short copy of the same ensemble (not timed).
        with lbl.Pool(64 << 30) as pool:
            for p, _ in reqs:
                pool.submit(p, init, 1000)
            pool.run(0)
            t = autotune.tune_pool(pool, "ensemble96/D2Q9/FD/%s" % (
                "fp32" if precision else "fp64"), steps=8)
            res["schedule"] = t["schedule"]
    with lbl.Pool(64 << 30) as pool:
        if tune:
            pool.set_schedule(**res["schedule"])
        ids = [pool.submit(p, init, nsteps) for p, _ in reqs]
        pool.run(0)  # admission: create and initialise every replica (not timed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pending = len(ids)
        while pending:
            pending = pool.run(tick)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        states = [pool.poll(i)[0] for i in ids]
        drift = 0.0
        for i in ids:
            tot = pool.result(i, lbl.LBL_RES_TOTALS)
            drift = max(drift, abs(tot[10] - tot[0]) / max(abs(tot[0]), 1e-300))
        res["schedule"] = pool.schedule()
    res.update({"seconds": round(dt, 4), "mlups": round(sites * nsteps / dt / 1e6, 1),
                "all_done": all(st == lbl.LBL_REQ_DONE for st in states),
                "max_mass_drift_rel": drift})
    return res


def served_mix(rate, seconds, seed=1234):
    """Poisson arrivals: (arrival time, kind) with 70% D2Q9 (side 64-512) and
    30% D3Q19 (side 64-192), one- or two-phase and FP32 or FP64 with
    probability 1/2 each, steps log-uniform in [500, 20000]."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t > seconds:
            break
        d3 = rng.random() < 0.3
        side = int(rng.integers(64, 193)) if d3 else int(rng.integers(64, 513))
        two_phase = rng.random() < 0.5
        fp32 = rng.random() < 0.5
        steps = int(round(math.exp(rng.uniform(math.log(500), math.log(20000)))))
        out.append({"t": t, "d3": d3, "side": side, "two_phase": two_phase, "fp32": fp32,
                    "steps": steps})
    return out


def run_served(lbl, torch, rate, seconds, budget_gb=200, tick=200, seed=1234):
    """Real-time serving loop over a pool: requests are submitted when their
    arrival time has passed, every tick advances all resident requests by up
    to `tick` steps, finished ones return S(k) and totals and are released.
    Latency = completion (end of the tick that finished it) - arrival."""
    import numpy as np
    mix = served_mix(rate, seconds, seed)
    lat, lups, drift = [], 0.0, 0.0
    max_queued = max_running = 0
    with lbl.Pool(int(budget_gb * 1e9)) as pool:
        live = {}
        nxt = 0
        t_start = time.monotonic()
        while nxt < len(mix) or live:
            now = time.monotonic() - t_start
            while nxt < len(mix) and mix[nxt]["t"] <= now:
                r = mix[nxt]
                i = nxt
                nxt += 1
                if r["two_phase"]:
                    a, b, init = -0.04, 0.04, lbl.make_init(kind=1, psi_std=1e-3)
                else:
                    a, b, init = 0.04, 0.1, lbl.make_init(kind=0, psi_std=1e-3)
                shape = (r["side"],) * 3 if r["d3"] else (r["side"], r["side"], 1)
                p = lbl.make_params(
                    lattice=lbl.LBL_D3Q19 if r["d3"] else lbl.LBL_D2Q9,
                    smol=lbl.LBL_SMOL_FV if r["d3"] else lbl.LBL_SMOL_FD,
                    precision=1 if r["fp32"] else 0, shape=shape, rho=1.0, eta=0.1, M=0.1,
                    a=a, b=b, kappa=0.05, kT=1e-5, seed=seed + i)
                rid = pool.submit(p, init, r["steps"])
                live[rid] = (r, shape[0] * shape[1] * shape[2])
            if not live:
                time.sleep(min(0.01, max(0.0, mix[nxt]["t"] - now)))
                continue
            pool.run(tick)
            t_end = time.monotonic() - t_start
            st_ = pool.stats()
            max_queued = max(max_queued, int(st_["queued"]))
            max_running = max(max_running, int(st_["running"]))
            for rid in list(live):
                st, _ = pool.poll(rid)
                if st in (lbl.LBL_REQ_DONE, lbl.LBL_REQ_FAILED):
                    r, n = live.pop(rid)
                    if st == lbl.LBL_REQ_DONE:
                        lat.append(t_end - r["t"])
                        lups += n * r["steps"]
                        pool.result(rid, lbl.LBL_RES_SK_AXES)
                        tot = pool.result(rid, lbl.LBL_RES_TOTALS)
                        drift = max(drift, abs(tot[10] - tot[0]) / max(abs(tot[0]), 1e-300))
                    pool.release(rid)
        t_total = time.monotonic() - t_start
        info = pool.stats()
    lat = np.array(lat) if lat else np.zeros(1)
    return {"rate_per_s": rate, "window_s": seconds, "requests": len(mix),
            "completed": int(len(lat)) if len(mix) else 0, "failed": int(info["failed"]),
            "p50_s": round(float(np.percentile(lat, 50)), 3),
            "p99_s": round(float(np.percentile(lat, 99)), 3),
            "aggregate_mlups": round(lups / t_total / 1e6, 1), "wall_s": round(t_total, 2),
            "budget_gb": budget_gb, "max_mass_drift_rel": drift,
            "max_queued": max_queued, "max_running": max_running,
            "mix": "70% D2Q9+FD side U{64..512}, 30% D3Q19+FV side U{64..192}; one/two-phase, "
                   "FP32/FP64 50/50; steps log-uniform [500, 20000]; S(k) and totals returned"}


def leg_error_vs_oracle(lbl, w, shape=None, nsteps=20):
    """Error against the FP64 oracle of a leg's kind of run (lattice, variant,
    options, parameters, initial state and seed as in the leg) on a smaller
    lattice: `nsteps` steps on the GPU in FP64 and in FP32-deviation storage,
    every site compared with the oracle's run of the same steps."""
    import numpy as np
    import oracle as O
    if shape is None:
        shape = (61, 47, 1) if w["lattice"] == 9 else (41, 37, 33)
    uw = w.get("u_wall", ((0, 0, 0), (0, 0, 0)))
    op = O.make_params(lattice=w["lattice"], smol=w["smol"], shape=shape, eta=w["eta"], M=w["M"],
                       a=w["a"], b=w["b"], kappa=w["kappa"], kT=w["kT"], seed=1234,
                       fd_noise=w.get("fd_noise", 0), force_form=w.get("force_form", 0),
                       walls=w.get("walls", 0), u_wall=tuple(uw[0]) + tuple(uw[1]))
    f, psi = O.init(op, w["init"], w["psi_std"])
    O.run(op, f, psi, 0, nsteps)
    out = {"shape": list(shape), "steps": nsteps,
           "measure": "max |gpu - oracle| / max |oracle| over all sites",
           "bound": {"fp64": 1e-12, "fp32dev": 1e-5}}
    for prec, name in ((0, "fp64"), (1, "fp32dev")):
        p = make_sim_params(lbl, dict(w, shape=shape), prec)
        with lbl.Sim(p, lbl.make_init(kind=w["init"], psi_std=w["psi_std"])) as sim:
            sim.step(nsteps)
            fg, pg = sim.observe(lbl.LBL_OBS_POP), sim.observe(lbl.LBL_OBS_PSI)
        out[name] = {"psi": float(np.abs(pg - psi).max() / np.abs(psi).max()),
                     "pop": float(np.abs(np.reshape(fg, f.shape) - f).max() / np.abs(f).max())}
    return out


def pool_error_vs_oracle(lbl, kinds, nsteps=100):
    """Error against the FP64 oracle of pooled requests: one request of each
    kind (lattice, variant, phase, storage) at the kind's smallest side runs
    `nsteps` steps in a pool and its psi is compared with the oracle's over the
    same steps.  A pooled request's fields are bitwise the same alone and in a
    mix (tested), so this is the error of every request of the kind."""
    import numpy as np
    import oracle as O
    out = []
    refs = {}
    for k in kinds:
        okey = (k["lattice"], k["smol"], k["shape"], k["two_phase"])
        a, b = (-0.04, 0.04) if k["two_phase"] else (0.04, 0.1)
        init = 1 if k["two_phase"] else 0
        if okey not in refs:
            p = O.make_params(lattice=k["lattice"], smol=k["smol"], shape=k["shape"], a=a, b=b,
                              kappa=0.05, M=0.1, kT=1e-5, eta=0.1, seed=k["seed"])
            f, psi = O.init(p, init, 1e-3)
            O.run(p, f, psi, 0, nsteps)
            refs[okey] = psi
        psi_ref = refs[okey]
        p = lbl.make_params(lattice=k["lattice"], smol=k["smol"], precision=k["precision"],
                            shape=k["shape"], rho=1.0, eta=0.1, M=0.1, a=a, b=b, kappa=0.05,
                            kT=1e-5, seed=k["seed"])
        with lbl.Pool(8 << 30) as pool:
            rid = pool.submit(p, lbl.make_init(kind=init, psi_std=1e-3), nsteps, keep_psi=True)
            while pool.run(50) > 0:
                pass
            psi = pool.result(rid, lbl.LBL_RES_PSI)
        err = float(np.abs(psi - psi_ref).max() / np.abs(psi_ref).max())
        out.append({"lattice": "D2Q9" if k["lattice"] == 9 else "D3Q19",
                    "smol": "FD" if k["smol"] == 0 else "FV", "shape": list(k["shape"]),
                    "two_phase": k["two_phase"],
                    "storage": "fp64" if k["precision"] == 0 else "fp32-deviation",
                    "steps": nsteps, "psi_rel_err": err,
                    "bound": 1e-12 if k["precision"] == 0 else 1e-5})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-plan", action="store_true",
                    help="skip the oracle timings of the 64^2 and 128^3 workloads")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-fp32", action="store_true",
                    help="skip the FP32-deviation run of the same lattice")
    ap.add_argument("--no-fd-noise", action="store_true",
                    help="skip the FD variant of the same lattice (link vs Fourier noise)")
    ap.add_argument("--no-stress", action="store_true",
                    help="skip the run of the same workload with the stress-divergence force")
    ap.add_argument("--no-walls", action="store_true",
                    help="skip the leg with sliding walls across the last axis")
    ap.add_argument("--no-slab", action="store_true",
                    help="skip the leg on one GPU's share of an 8-way z-slab decomposition")
    ap.add_argument("--no-tune", action="store_true", help="no autotuning of the pool legs")
    ap.add_argument("--tune-single", action="store_true",
                    help="autotune the single-run schedule too (default: the library's own)")
    ap.add_argument("--schedule", default=None,
                    help="fix the single-run schedule as lb_width,xcd_swizzle,zc (no tuning)")
    ap.add_argument("--ensemble-steps", type=int, default=5000)
    ap.add_argument("--serve-rate", type=float, default=20.0,
                    help="Poisson arrival rate (requests/s) of the served mix (20/s)")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="arrival window (s); the full mix is 300 s")
    ap.add_argument("--sub-rate", type=float, default=2.0,
                    help="a second served run below saturation (0: skip)")
    ap.add_argument("--sub-seconds", type=float, default=10.0)
    ap.add_argument("--bound-budget-gb", type=float, default=6.0,
                    help="a served run of the same arrivals under this HBM budget (0: skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 2 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1104_0078_amd import lbl

    if args.calibrate_copy:
        n = (2 << 30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_each_way": n * 8, "launches": 5}))
        return

    tune = not args.no_tune
    fixed = None
    if args.schedule:
        lw_, sw_, zc_ = (int(v) for v in args.schedule.split(","))
        fixed = dict(lb_width=lw_, xcd_swizzle=sw_, zc=zc_)
    w = WORKLOADS[args.workload]
    r = run_single(lbl, torch, w, args.workload, args.steps, args.warmup, args.tune_single,
                   schedule=fixed)
    N = r["N"]
    print("single run done: %.1f MLUPS" % r["mlups"], file=sys.stderr, flush=True)
    # Per-kernel HBM roofline from the event timings; the dominant kernel is
    # the one with the largest share of device time.
    per_kernel = {}
    for kname, klaunch, kms in r["ktimes"]:
        avg_s = kms / klaunch / 1e3
        kb = kernel_alg_bytes_per_site(kname, w, schedule=r["schedule"])
        if kb is None:
            continue
        achieved = kb * N / avg_s / 1e9
        traffic = traffic_for(kname, args.workload)
        per_kernel[kname] = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(achieved / HBM_PEAK_GBS, 4),
                             "traffic": traffic,
                             # the measured HBM bytes moved at this launch time
                             "traffic_gbs": (round(traffic / avg_s / 1e9, 1)
                                             if traffic is not None else None),
                             "avg_launch_ms": round(avg_s * 1e3, 4), "launches": klaunch,
                             "alg_bytes_per_site": kb}
    # Headline roofline: the dominant kernel (largest share of device time),
    # its algorithmic bytes being its share of the step's state bytes (the
    # populations it reads and writes once), over its mean launch time from
    # the HIP events of the timed region; beside it the whole step, 2 Q b +
    # 2 b per site over the step time, and the step's measured HBM traffic.
    dom_t = max(r["ktimes"], key=lambda t: t[2])
    dom = dom_t[0]
    sb = state_bytes_per_site(dom, w)
    step_frac = r["mlups"] * 1e6 * alg_bytes_per_site(w) / (HBM_PEAK_GBS * 1e9)
    step_traffic = step_traffic_per_site(r["ktimes"], args.workload, args.steps, N)
    roofline = None
    if sb is not None:
        avg_s = dom_t[2] / dom_t[1] / 1e3
        achieved = sb * N / avg_s / 1e9
        traffic = traffic_for(dom, args.workload)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "traffic_gbs": (round(traffic / avg_s / 1e9, 1)
                                    if traffic is not None else None),
                    "avg_launch_ms": round(avg_s * 1e3, 4), "launches": dom_t[1],
                    "alg_bytes_per_site": sb,
                    "alg_bytes_meaning": "populations read and written once (2Qb), the "
                                         "kernel's share of the 2Qb + 2b state bytes"}
    step_roofline = {"alg_bytes_per_site": alg_bytes_per_site(w),
                     "achieved": round(alg_bytes_per_site(w) * r["mlups"] * 1e6 / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(step_frac, 4),
                     "traffic_bytes_per_site": (round(step_traffic, 1)
                                                if step_traffic is not None else None)}
    if roofline is not None:
        roofline["step"] = step_roofline
    out = {
        "metric": METRIC,
        "value": round(r["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w["precision"] == 0 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": "D2Q9" if w["lattice"] == 9 else "D3Q19",
                   "smol": "FD" if w["smol"] == 0 else "FV",
                   "storage": "fp64" if w["precision"] == 0 else "fp32-deviation",
                   "shape": list(w["shape"]), "sites": N, "global_batch": 1,
                   "parallelism": "single GPU", "schedule": r["schedule"]},
        "hbm_alg_frac_step": round(step_frac, 4),
        "alg_bytes_per_site_step": alg_bytes_per_site(w),
        "traffic_bytes_per_site_step": step_roofline["traffic_bytes_per_site"],
        "roofline": roofline if roofline is not None else step_roofline,
        # kernel level: every field a kernel reads or writes counted once
        "kernel_rooflines": {k: {"frac": v["frac"], "achieved": v["achieved"],
                                 "alg_bytes_per_site": v["alg_bytes_per_site"],
                                 "traffic_gbs": v["traffic_gbs"],
                                 "avg_launch_ms": v["avg_launch_ms"]}
                             for k, v in per_kernel.items()},
        "kernels_ms_per_step": {t[0]: round(t[2] / max(1, args.steps), 4) for t in r["ktimes"]},
        "mass_total": r["totals"][0],
    }
    if w["precision"] == 0 and not args.no_fp32:
        r32 = run_single(lbl, torch, w, args.workload, args.steps, args.warmup,
                         args.tune_single, precision=1)
        out["fp32dev_same_lattice"] = {"value": round(r32["mlups"], 2), "unit": "MLUPS",
                                       "ms_per_step": round(r32["ms_per_step"], 4),
                                       "schedule": r32["schedule"]}
        print("fp32 run done: %.1f MLUPS" % r32["mlups"], file=sys.stderr, flush=True)
    if not args.no_fd_noise:
        # The FD variant of the same workload with its conserved noise built
        # both ways: link fluxes in-kernel, and the paper's Fourier-space
        # construction (a hipFFT pair per step).
        legs = {}
        for fdn, name in ((0, "link"), (1, "fourier")):
            wf = dict(w, smol=0, fd_noise=fdn)
            rf = run_single(lbl, torch, wf, args.workload, min(args.steps, 30), args.warmup, False)
            legs[name] = {"value": round(rf["mlups"], 2), "unit": "MLUPS",
                          "ms_per_step": round(rf["ms_per_step"], 4),
                          "kernels_ms_per_step": {t[0]: round(t[2] / min(args.steps, 30), 4)
                                                  for t in rf["ktimes"]},
                          "error_vs_oracle": leg_error_vs_oracle(lbl, wf)}
        out["fd_noise_same_lattice"] = legs
        print("fd noise legs done: link %.1f, Fourier %.1f MLUPS" % (
            legs["link"]["value"], legs["fourier"]["value"]), file=sys.stderr, flush=True)
    if not args.no_stress:
        # The same workload with the force as the divergence of the stress of
        # Eq. (muf) (momentum conserved exactly; two more per-site passes).
        nst = min(args.steps, 30)
        rs_ = run_single(lbl, torch, dict(w, force_form=1), args.workload, nst, args.warmup, False)
        out["stress_force_same_workload"] = {
            "value": round(rs_["mlups"], 2), "unit": "MLUPS",
            "ms_per_step": round(rs_["ms_per_step"], 4),
            "kernels_ms_per_step": {t[0]: round(t[2] / nst, 4) for t in rs_["ktimes"]},
            "error_vs_oracle": leg_error_vs_oracle(lbl, dict(w, force_form=1))}
        print("stress force leg done: %.1f MLUPS" % rs_["mlups"], file=sys.stderr, flush=True)
    if not args.no_walls and w["smol"] == 1:
        # The same workload between walls across the last axis sliding at
        # (0.02, -0.01, 0) and (-0.015, 0.01, 0): bounce-back LB passes and
        # the wall stencils (per-site kernels).
        nw = min(args.steps, 30)
        ww = dict(w, walls=1, u_wall=((0.02, -0.01, 0.0), (-0.015, 0.01, 0.0)))
        rw = run_single(lbl, torch, ww, args.workload, nw, args.warmup, False)
        out["walls_same_workload"] = {
            "value": round(rw["mlups"], 2), "unit": "MLUPS",
            "ms_per_step": round(rw["ms_per_step"], 4),
            "kernels_ms_per_step": {t[0]: round(t[2] / nw, 4) for t in rw["ktimes"]},
            "error_vs_oracle": leg_error_vs_oracle(lbl, ww)}
        print("walls leg done: %.1f MLUPS" % rw["mlups"], file=sys.stderr, flush=True)
    if not args.no_slab and w["lattice"] != 9 and w["shape"][2] % 8 == 0:
        # One GPU's share of the same lattice split into 8 z-slabs: the step
        # on nx x ny x nz/8 sites (periodic along z standing in for the halo
        # exchange, which is not run).
        nsl = min(args.steps, 30)
        ws = dict(w, shape=(w["shape"][0], w["shape"][1], w["shape"][2] // 8))
        rsl = run_single(lbl, torch, ws, args.workload, nsl, args.warmup, False)
        out["shard_slab_one_gpu"] = {
            "shape": list(ws["shape"]), "value": round(rsl["mlups"], 2), "unit": "MLUPS",
            "ms_per_step": round(rsl["ms_per_step"], 4),
            "kernels_ms_per_step": {t[0]: round(t[2] / nsl, 4) for t in rsl["ktimes"]},
            "note": "one GPU's share of an 8-way z-slab decomposition; periodic along z "
                    "in place of the halo exchange, which is not run"}
        print("slab leg done: %.1f MLUPS" % rsl["mlups"], file=sys.stderr, flush=True)
    if not args.no_batched:
        out["batched"] = {}
        for prec, name in ((1, "fp32"), (0, "fp64")):
            out["batched"][name] = run_ensemble(lbl, torch, prec, args.ensemble_steps, tune)
            print("ensemble %s done: %.1f MLUPS" % (name, out["batched"][name]["mlups"]),
                  file=sys.stderr, flush=True)
        # the ensemble's kind: D2Q9 + FD one-phase, replica 0's seed, smallest side
        out["batched"]["error_vs_oracle"] = pool_error_vs_oracle(lbl, [
            dict(lattice=9, smol=0, shape=(32, 32, 1), two_phase=False, precision=pr,
                 seed=1234) for pr in (0, 1)])
    if not args.no_served:
        # At the mix's own arrival rate (overloaded: the offered load exceeds
        # the device, so latency includes the queue), then below saturation.
        out["served"] = run_served(lbl, torch, args.serve_rate, args.serve_seconds)
        if args.serve_rate != 20.0 or args.serve_seconds != 300.0:
            out["served"]["sample"] = ("bounded sample of the 20/s x 300 s mix (rate %.3g/s, "
                                       "window %.3g s)" % (args.serve_rate, args.serve_seconds))
        print("served done: p50 %.2f s p99 %.2f s, %.0f MLUPS" % (
            out["served"]["p50_s"], out["served"]["p99_s"], out["served"]["aggregate_mlups"]),
              file=sys.stderr, flush=True)
        # The same arrivals with an HBM budget that binds: requests wait in
        # the queue until resident ones finish and release their memory.
        if args.bound_budget_gb > 0:
            bb = run_served(lbl, torch, args.serve_rate, args.serve_seconds,
                            budget_gb=args.bound_budget_gb)
            bb["sample"] = ("bounded sample of the mix (rate %.3g/s, window %.3g s) under an "
                            "HBM budget of %g GB" % (args.serve_rate, args.serve_seconds,
                                                     args.bound_budget_gb))
            out["served_budget_bound"] = bb
            print("served (budget %g GB) done: p50 %.2f s p99 %.2f s, max queued %d" % (
                args.bound_budget_gb, bb["p50_s"], bb["p99_s"], bb["max_queued"]),
                  file=sys.stderr, flush=True)
        # one request of every kind of the mix against the oracle
        kinds = [dict(lattice=lat, smol=sm, shape=shp, two_phase=tp, precision=pr, seed=1234)
                 for lat, sm, shp in ((9, 0, (64, 64, 1)), (19, 1, (64, 64, 64)))
                 for tp in (False, True) for pr in (0, 1)]
        out["served"]["error_vs_oracle"] = pool_error_vs_oracle(lbl, kinds)
        print("served error vs oracle done", file=sys.stderr, flush=True)
        if args.sub_rate > 0:
            sub = run_served(lbl, torch, args.sub_rate, args.sub_seconds)
            sub["sample"] = "below saturation (rate %.3g/s, window %.3g s)" % (
                args.sub_rate, args.sub_seconds)
            out["served_below_saturation"] = sub
            print("served (below saturation) done: p50 %.2f s p99 %.2f s" % (
                sub["p50_s"], sub["p99_s"]), file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.workload, lbl=lbl)
        out["cpu_baseline"]["cpu_model"] = cpu_model()
        out["cpu_baseline"]["host_threads"] = os.cpu_count()
        if not args.no_cpu_plan:
            out["cpu_baseline"]["specified_workloads"] = cpu_baseline_plan(lbl, torch)
            print("cpu baseline of the specified workloads done", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
