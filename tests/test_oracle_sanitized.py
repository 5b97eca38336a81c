"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
only) and driven through every lattice, variant, coupling and stage count on
small odd lattices (tests/oracle_sanitize_driver.c): no out-of-bounds access,
leak or undefined behaviour may be reported."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitized")
    cmd = [gcc, "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", os.path.join(ROOT, "oracle"), os.path.join(ROOT, "oracle", "lbl_oracle.c"),
           os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"), "-o", exe, "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0 and "clean" in run.stdout, run.stdout + run.stderr
