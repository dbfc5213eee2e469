"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sparc_oracle.c is compiled together with tests/oracle_sanitize_driver.c
(gcc, -fsanitize=address,undefined, every report fatal) and run: each entry
point on grids smaller than the stencil, both boundary modes, projector cubes
at both walls and padded leading dimensions, plus two checks any correct
operator passes (H symmetric, degree-1 filter = (sigma_1/e)(H - c) X).  The
build goes to tests/_build (ignored by git); OpenMP is left out so that the
run is the serial code path, free of the OpenMP runtime's own allocations."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "sparc_oracle.c")
DRIVER = os.path.join(HERE, "oracle_sanitize_driver.c")
BUILD = os.path.join(HERE, "_build")

SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_and_ubsan():
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "oracle_sanitized")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-Wall", *SAN_FLAGS, "-o", exe, SRC, DRIVER, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("asan" in r.stderr.lower() or "ubsan" in r.stderr.lower()):
        pytest.skip("sanitizer runtimes not installed: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-4000:]
    assert "oracle sanitizer driver: ok" in r.stdout
