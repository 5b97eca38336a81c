"""Launch-schedule autotuner for the sweep.

A schedule changes only speed, never results (the fields are bitwise the same
under every schedule), so candidates are timed on live work: a simulation is
advanced a few steps under each candidate with the library's per-kernel HIP
event timers, a pool ticks its resident requests under each candidate.  The
fastest candidate is kept and stored in a JSON cache keyed by what decides the
kernels' shape (lattice, SMOL variant, storage, lattice sides, or a pool's
request mix), so the next run starts from it without timing again.

Schedule knobs (see lbl_set_schedule / lbl_pool_set_schedule in lbl.h):
  lb_width     sites along x per 256-thread block of the per-site LB kernels;
  xcd_swizzle  block order that hands each XCD a contiguous part of the work
               (single simulations: bit 0 the LB kernels, bit 1 the SMOL tiles);
  zc           planes per block of the z-marching SMOL kernels (3-D);
  overlap      1: the first stage, 2: the SMOL noise on a second stream,
               3: the SMOL noise inside the velocity pass (the default), 0: none
               (single simulations).
"""
import json
import os
import time

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1104_0078_amd",
                             "schedules.json")


def cache_path():
    return os.environ.get("LBL_TUNE_CACHE", DEFAULT_CACHE)


def _load(path):
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path, key, entry):
    data = _load(path)
    data[key] = entry
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def sim_key(params):
    return "sim/Q%d/%s/%s/%dx%dx%d/rk%d" % (
        params.lattice, "FV" if params.smol else "FD", "fp32" if params.precision else "fp64",
        params.nx, params.ny, params.nz, params.rk_stages)


def sim_candidates(params, overlap=0):
    widths = [w for w in (32, 64, 128, 256) if w <= max(32, params.nx)]
    widths = widths[-3:]
    zcs = [0]  # 0: the library's per-kernel defaults (from occupancy)
    if params.nz > 1:
        zcs = [0] + sorted({z for z in (8, 16, 32, 64) if z <= params.nz} or {params.nz})
    swz = (0, 1, 2, 3) if params.nz > 1 else (0, 1)
    return [dict(lb_width=w, xcd_swizzle=s, zc=z, overlap=overlap) for w in widths for s in swz
            for z in zcs]


def _time_sim(sim, cand, steps):
    """Wall time per step of `steps` steps under one schedule (host clock
    around the synchronised batch, so concurrent streams count once)."""
    import torch
    sim.set_schedule(**cand)
    sim.step(1)  # first launch of a shape outside the timing
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def tune_sim(sim, params, steps=6, use_cache=True, candidates=None):
    """Pick the fastest schedule for a live simulation and apply it.  Returns
    {"schedule": ..., "ms_per_step": ..., "from_cache": bool, "table": [...]}.
    The steps taken while timing are real steps of the simulation."""
    path = cache_path()
    key = sim_key(params)
    if use_cache:
        hit = _load(path).get(key)
        if hit:
            sim.set_schedule(**hit["schedule"])
            return dict(hit, from_cache=True)
    table = []
    ov0 = sim.schedule()["overlap"]  # the library's default for this lattice
    sim.step(8)  # clocks and caches settle before the first candidate
    for cand in candidates or sim_candidates(params, ov0):
        table.append({"schedule": cand, "ms_per_step": round(_time_sim(sim, cand, steps), 4)})
    best = min(table, key=lambda r: r["ms_per_step"])
    # Last dimension, on top of the best schedule so far: the first stage on
    # a second stream, concurrent with the velocity pass (full coupling,
    # several stages), the SMOL noise on it, concurrent with the LB passes,
    # the noise inside the velocity pass (the default), or none of these.
    overlaps = [0]
    if params.coupling == 0 and params.rk_stages > 1:
        overlaps.append(1)
    if params.coupling != 2 and params.kT > 0:
        overlaps.append(2)
    if ov0 == 3:
        overlaps.append(3)
    base = best["schedule"]
    for ov in overlaps:
        if ov == base["overlap"]:
            continue
        cand = dict(base, overlap=ov)
        table.append({"schedule": cand, "ms_per_step": round(_time_sim(sim, cand, steps), 4)})
    best = min(table, key=lambda r: r["ms_per_step"])
    sim.set_schedule(**best["schedule"])
    entry = {"schedule": best["schedule"], "ms_per_step": best["ms_per_step"], "table": table}
    _store(path, key, entry)
    return dict(entry, from_cache=False)


def pool_candidates(has_3d):
    zcs = (0, 8, 16) if has_3d else (0,)
    return [dict(lb_width=w, xcd_swizzle=s, zc=z) for w in (64, 128, 256) for s in (0, 1)
            for z in zcs]


def tune_pool(pool, key, steps=8, has_3d=False, use_cache=True, candidates=None):
    """Pick the fastest work-table schedule for the requests resident in a pool
    (ticking them under each candidate) and apply it.  `key` names the request
    mix for the cache.  Each candidate takes two ticks of `steps` steps (the
    first rebuilds the tables and captures the graph, the second is timed), so
    the resident requests need that many steps left."""
    import torch
    path = cache_path()
    full_key = "pool/" + key
    if use_cache:
        hit = _load(path).get(full_key)
        if hit:
            pool.set_schedule(**hit["schedule"])
            return dict(hit, from_cache=True)
    table = []
    for cand in candidates or pool_candidates(has_3d):
        pool.set_schedule(**cand)
        pool.run(steps)  # rebuild the tables and capture the tick outside the timing
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pool.run(steps)
        torch.cuda.synchronize()
        table.append({"schedule": cand,
                      "ms_per_step": round((time.perf_counter() - t0) * 1e3 / steps, 4)})
    best = min(table, key=lambda r: r["ms_per_step"])
    pool.set_schedule(**best["schedule"])
    entry = {"schedule": best["schedule"], "ms_per_step": best["ms_per_step"], "table": table}
    _store(path, full_key, entry)
    return dict(entry, from_cache=False)
