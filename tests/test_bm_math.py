"""Host check of the elementary functions behind the GPU sweep's Box-Muller
normals (paper_1104_0078_amd/csrc/lbl_math.hpp): on the exact argument set
u = (k + 1/2) 2^-32 they must agree with extended-precision libm to a few
units of 2^-52, so the FP64 normals agree with the oracle's to rounding."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("bm") / "bm_math_check")
    cmd = [hipcc, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1104_0078_amd", "csrc"),
           os.path.join(ROOT, "tests", "bm_math_check.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    return exe


def test_box_muller_functions_accuracy(checker):
    out = subprocess.run([checker, "1000000"], capture_output=True, text=True, check=True).stdout
    vals = {line.split()[0]: float(line.split()[1]) for line in out.strip().splitlines()}
    print(out)
    assert vals["log_rel_ulp"] < 4.0
    assert vals["sin_abs_ulp"] < 2.0
    assert vals["cos_abs_ulp"] < 2.0
    assert vals["pyth_ulp"] < 4.0
