"""Pins of the oracle's noise generator (Philox4x32-10 + Box-Muller).

The paper fixes only that the noises are zero-mean Gaussian white noises with
the variances of Eqs. (fdt_orderpara) and (stressfdt); the generator is this
project's choice.  It is pinned against (1) the known-answer vectors published
with Random123 (tests/golden/philox4x32_10_kat.txt), (2) rocRAND's independent
implementation, and (3) the moments of the standard normal law.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, expect in rows:
        assert O.philox(ctr, key) == expect


@pytest.mark.skipif(not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h")
                    or shutil.which("g++") is None, reason="rocRAND headers or g++ missing")
def test_philox_matches_rocrand(tmp_path):
    exe = tmp_path / "ref"
    subprocess.run(["g++", "-O1", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__",
                    os.path.join(HERE, "rocrand_philox_ref.cpp"), "-o", str(exe)], check=True)
    rng = np.random.default_rng(7)
    q = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    text = "\n".join(" ".join("%08x" % int(v) for v in row) for row in q) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True)
    ref = [[int(t, 16) for t in line.split()] for line in out.stdout.strip().splitlines()]
    assert len(ref) == len(q)
    for row, r in zip(q, ref):
        assert O.philox(row[:4], row[4:]) == r


def test_normal_moments():
    # 4 slots x 40000 sites: mean 0, variance 1, kurtosis 3, no lane correlation.
    z = np.array([[O.normal(99, s, 3, O.TAG_LB, slot) for slot in range(4)]
                  for s in range(40000)])
    n = z.shape[0]
    assert np.all(np.abs(z.mean(axis=0)) < 5 / np.sqrt(n))
    assert np.all(np.abs(z.var(axis=0) - 1) < 5 * np.sqrt(2 / n))
    assert np.all(np.abs((z ** 4).mean(axis=0) - 3) < 5 * np.sqrt(96 / n))
    c = np.corrcoef(z.T)
    assert np.abs(c - np.eye(4)).max() < 5 / np.sqrt(n)


def test_normal_box_muller_mapping():
    # Lanes 0/1 share a radius, and lane 1 is the sine partner of lane 0.
    ctr_key = lambda s, st, blk, tag, seed: ([s, st, blk, tag], [seed & 0xFFFFFFFF, seed >> 32])
    seed = (5 << 32) | 17
    for s in range(50):
        x = O.philox(*ctr_key(s, 11, 1, O.TAG_SMOL, seed))
        u = [(v + 0.5) * 2.0 ** -32 for v in x]
        r0 = np.sqrt(-2 * np.log(u[0]))
        r1 = np.sqrt(-2 * np.log(u[2]))
        expect = [r0 * np.cos(2 * np.pi * u[1]), r0 * np.sin(2 * np.pi * u[1]),
                  r1 * np.cos(2 * np.pi * u[3]), r1 * np.sin(2 * np.pi * u[3])]
        got = [O.normal(seed, s, 11, O.TAG_SMOL, 4 + lane) for lane in range(4)]
        np.testing.assert_allclose(got, expect, rtol=1e-14, atol=1e-14)


def test_normals_distinct_streams():
    # Different tags, steps, sites and seeds give different numbers.
    base = O.normal(1, 10, 20, 0, 0)
    for args in [(2, 10, 20, 0, 0), (1, 11, 20, 0, 0), (1, 10, 21, 0, 0), (1, 10, 20, 1, 0),
                 (1, 10, 20, 0, 1)]:
        assert O.normal(*args) != base
