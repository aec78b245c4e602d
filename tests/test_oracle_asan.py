"""The oracle's pins under the address and undefined-behaviour checkers: a
CPU build of the oracle's C sources (collision, sedimentation,
condensation) with -fsanitize=address,undefined (no
recovery), loaded into a Python process that preloads the checker runtime,
runs the oracle's pin suites; any out-of-bounds access, use after free,
leak-free misuse or undefined arithmetic aborts that process."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    r = subprocess.run(["gcc", "-print-file-name=" + name],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) else None


@pytest.mark.slow
def test_oracle_pins_under_address_and_ub_checkers():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc address-checker runtime not found")
    env = dict(os.environ)
    env["FSBM_ORACLE_SANITIZE"] = "1"
    env["LD_PRELOAD"] = asan
    # CPython's own allocations are not ours to check for leaks
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["OMP_NUM_THREADS"] = "4"
    cmd = [sys.executable, "-c",
           "import oracle; oracle.build(force=True)"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu",
           "-p", "no:cacheprovider",
           "tests/test_oracle_pins.py", "tests/test_oracle_sequential.py",
           "tests/test_oracle_sed.py", "tests/test_oracle_cond.py"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out
    assert "runtime error" not in out
    assert "passed" in out
