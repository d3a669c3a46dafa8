"""The C oracle built with AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only) and driven by
tests/oracle_sanitize_main.c: random inputs for every d from 1 to 8, empty
and one-point sets, duplicates, coordinates at +-2^24, MinPts up to n + 1.
The run must report no sanitizer error, and the cell-based oracle must agree
with the all-pairs one and with Definition 1's neighbour counts."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-Wall", "-Wextra", "-Werror",
           os.path.join(ROOT, "oracle", "dbscan_oracle.c"), os.path.join(ROOT, "tests", "oracle_sanitize_main.c"),
           "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="4")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert "all agree" in r.stdout
