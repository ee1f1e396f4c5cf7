"""The oracle's C source under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only): it is rebuilt with both sanitizers into a temporary
library and the oracle's pins (tests/test_oracle_pins.py) run again, in a
child process with the sanitizer runtimes preloaded, against that build.  A
memory error or undefined behaviour anywhere the pins reach (the column
product, the merge sort, the transpose, the output buffers) aborts the
child."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def test_oracle_pins_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("sanitizer runtimes not installed")
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared",
                           "-fPIC", "-o", str(lib), os.path.join(ROOT, "oracle", "spgemm_oracle.c"), "-lm"])
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", PB_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    log = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, log
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, log
    assert " passed" in r.stdout, log
