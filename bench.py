"""Benchmark of the coupled FLBE + SMOL sweep on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

Prints ONE JSON line.  A "step" is one full coupled time step (LB collide and
stream with noise, chemical potential, force, SMOL Runge-Kutta with noise) over
the whole lattice, with the state already resident in HBM.  value = lattice
sites x steps / wall time of the timed region (MLUPS, million lattice-site
updates per second).  The kernel roofline figure is measured live with HIP
events on the library's stream during the same timed region.
"""
import argparse
import hashlib
import json
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


def kernel_alg_bytes_per_site(name, w, rk=2):
    """Algorithmic bytes per site of one launch of each kernel: the data the
    kernel must move at minimum.
      k_lb:    read and write the Q populations, read psi;
      k_prep:  read psi, write mu and the SMOL noise;
      k_stage: read the stage input, u (d values) and the noise, write the
               output; the final Heun stage also reads psi^n (per-launch mean)."""
    b = 8 if w["precision"] == 0 else 4
    d = 2 if w["lattice"] == 9 else 3
    if name.startswith("k_lb"):
        return 2 * w["lattice"] * b + b
    if name.startswith("k_prep"):
        return 3 * b
    if name.startswith("k_stage"):
        return (3 + d) * b + (b / 2 if rk == 2 else 0)
    return None


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1104_0078_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, fn), "rb") as fh:
            h.update(fn.encode())
            h.update(fh.read())
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


def cpu_baseline(w, workload_name):
    """The FP64 oracle, as it stands, on a bounded sample: one step of the same
    lattice (or a few on small lattices), timed on the host cores."""
    import numpy as np  # noqa: F401
    import oracle as O

    p = O.make_params(lattice=w["lattice"], smol=w["smol"], shape=w["shape"], a=w["a"],
                      b=w["b"], kappa=w["kappa"], M=w["M"], kT=w["kT"], eta=w["eta"],
                      seed=1234)
    f, psi = O.init(p, w["init"], w["psi_std"])
    N = O.nsites(p)
    nsteps = max(1, min(200, int(2e7 // N)))
    t0 = time.perf_counter()
    O.run(p, f, psi, 0, nsteps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": N * nsteps / dt / 1e6, "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "sample": "%d step(s) of %s (%d sites), FP64 oracle, %.1f s" % (
                nsteps, workload_name, N, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    w = WORKLOADS[args.workload]
    params = lbl.make_params(lattice=w["lattice"], smol=w["smol"], precision=w["precision"],
                             shape=w["shape"], rho=1.0, eta=w["eta"], M=w["M"], a=w["a"],
                             b=w["b"], kappa=w["kappa"], kT=w["kT"], seed=1234)
    init = lbl.make_init(kind=w["init"], psi_std=w["psi_std"])
    stream = torch.cuda.current_stream()
    N = w["shape"][0] * w["shape"][1] * w["shape"][2]
    with lbl.Sim(params, init, device=0, stream=stream) as sim:
        sim.step(args.warmup)
        torch.cuda.synchronize()
        sim.timing(True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        sim.step(args.steps)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        gpu_ms = ev0.elapsed_time(ev1)
        ktimes = sim.kernel_times()
        sim.timing(False)
        tot = sim.observe(lbl.LBL_OBS_TOTALS)
    seconds = max(wall, gpu_ms / 1e3)
    ms_per_step = seconds * 1e3 / args.steps
    mlups = N * args.steps / seconds / 1e6
    # Per-kernel HBM roofline from the event timings; the dominant kernel is
    # the one with the largest share of device time.
    per_kernel = {}
    for kname, klaunch, kms in ktimes:
        avg_s = kms / klaunch / 1e3
        kb = kernel_alg_bytes_per_site(kname, w)
        if kb is None:
            continue
        achieved = kb * N / avg_s / 1e9
        per_kernel[kname] = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(achieved / HBM_PEAK_GBS, 4),
                             "traffic": traffic_for(kname, args.workload),
                             "avg_launch_ms": round(avg_s * 1e3, 4), "launches": klaunch,
                             "alg_bytes_per_site": kb}
    dom = max(ktimes, key=lambda r: r[2])[0]
    roofline = per_kernel.get(dom)
    step_frac = mlups * 1e6 * alg_bytes_per_site(w) / (HBM_PEAK_GBS * 1e9)
    out = {
        "metric": METRIC,
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w["precision"] == 0 else "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": "D2Q9" if w["lattice"] == 9 else "D3Q19",
                   "smol": "FD" if w["smol"] == 0 else "FV",
                   "storage": "fp64" if w["precision"] == 0 else "fp32-deviation",
                   "shape": list(w["shape"]), "sites": N, "global_batch": 1,
                   "parallelism": "single GPU"},
        "hbm_alg_frac_step": round(step_frac, 4),
        "alg_bytes_per_site_step": alg_bytes_per_site(w),
        "roofline": roofline,
        "kernel_rooflines": {k: {"frac": v["frac"], "achieved": v["achieved"],
                                 "avg_launch_ms": v["avg_launch_ms"]}
                             for k, v in per_kernel.items()},
        "kernels_ms_per_step": {r[0]: round(r[2] / max(1, args.steps), 4) for r in ktimes},
        "mass_total": tot[0],
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.workload)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
