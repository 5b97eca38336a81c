"""Host-side checks of bench.py's contract (no GPU): the multi-GPU request is
refused with a message, and the algorithmic byte counts behind the roofline
fields are the ones the kernels' data movement gives."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_of_the_headline_workload():
    w = bench.WORKLOADS[bench.DEFAULT_WORKLOAD]
    assert w["lattice"] == 19 and w["precision"] == 0 and w["shape"] == (256, 256, 256)
    # state read and written once per step: 2 Q b + 2 b
    assert bench.alg_bytes_per_site(w) == 2 * 19 * 8 + 2 * 8 == 320
    # k_lb: Q pulls + Q writes + psi + mu + u^n (d = 3)
    assert bench.kernel_alg_bytes_per_site("k_lb", w) == (2 * 19 + 2 + 3) * 8 == 344
    # k_uend: Q pulls + psi + mu + the stage velocity
    assert bench.kernel_alg_bytes_per_site("k_uend", w) == (19 + 2 + 3) * 8
    assert bench.kernel_alg_bytes_per_site("k_prep", w) == 3 * 8
    assert bench.kernel_alg_bytes_per_site("k_stage", w) == (3 + 3) * 8 + 4
    # the default schedule of FV on 3-D lattices draws the noise in the
    # velocity pass: its b bytes move from the preparation kernel to it
    fused = {"overlap": 3}
    assert bench.kernel_alg_bytes_per_site("k_uend", w, schedule=fused) == (19 + 3 + 3) * 8
    assert bench.kernel_alg_bytes_per_site("k_prep", w, schedule=fused) == 2 * 8
    wfd = dict(w, smol=0)
    assert bench.kernel_alg_bytes_per_site("k_prep", wfd, schedule=fused) == 2 * 8
    # the noise built in Fourier space is drawn apart from both
    wff = dict(w, smol=0, fd_noise=1)
    assert bench.kernel_alg_bytes_per_site("k_prep", wff, schedule=fused) == 3 * 8
    assert bench.kernel_alg_bytes_per_site("k_uend", wff, schedule=fused) == (19 + 2 + 3) * 8
    w32 = dict(w, precision=1)
    assert bench.alg_bytes_per_site(w32) == 160
    assert bench.kernel_alg_bytes_per_site("k_white", w) is None
    # headline roofline: the LB pass's share of the state bytes, the populations
    assert bench.state_bytes_per_site("k_lb", w) == 2 * 19 * 8 == 304
    assert bench.state_bytes_per_site("k_lb", w32) == 2 * 19 * 4
    assert bench.state_bytes_per_site("k_stage", w) is None


def test_step_traffic_sums_the_kernels_of_a_step(monkeypatch):
    """The step's measured traffic per site is the sum over its kernels of
    the counter bytes per launch times launches per step, over N."""
    per_launch = {"k_lb": 4.0e9, "k_prep": 5.0e8, "k_stage": 1.5e9}
    monkeypatch.setattr(bench, "traffic_for", lambda k, wl: per_launch.get(k))
    kt = [("k_prep", 10, 3.3), ("k_lb", 10, 12.0), ("k_stage", 20, 5.6)]
    N = 256 ** 3
    got = bench.step_traffic_per_site(kt, "any", 10, N)
    assert abs(got - (4.0e9 + 5.0e8 + 2 * 1.5e9) / N) < 1e-9
    assert bench.step_traffic_per_site(kt + [("k_other", 10, 1.0)], "any", 10, N) is None


def test_committed_traffic_entries_are_self_consistent():
    """Each entry of profiles/traffic.json scales the counters by the copy
    calibration it records; the bench reports it only for matching sources."""
    import json
    entries = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert {e["kernel"] for e in entries} >= {"k_lb", "k_uend", "k_prep", "k_stage"}
    for e in entries:
        scaled = (e["fetch_kib"] * 1024 * e["fetch_factor"] + e["write_kib"] * 1024 *
                  e["write_factor"])
        assert abs(scaled / e["bytes_per_launch"] - 1) < 1e-12
        assert e["bytes_per_launch"] > e["alg_bytes_per_launch"] * 0.9


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    """The committed counter summary is keyed by a hash of the kernel sources
    without comments: a comment edit keeps it, a code edit drops it."""
    import shutil
    src = os.path.join(ROOT, "paper_1104_0078_amd", "csrc")
    dst = tmp_path / "paper_1104_0078_amd" / "csrc"
    shutil.copytree(src, dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.source_hash()
    k = dst / "lbl_kernels.hpp"
    text = k.read_text()
    k.write_text("// an added line comment\n/* and a block\n   comment */\n" +
                 text.replace(";", ";  // trailing comment", 1))
    assert bench.source_hash() == h0
    k.write_text(text + "\nstatic int added_code;\n")
    assert bench.source_hash() != h0
