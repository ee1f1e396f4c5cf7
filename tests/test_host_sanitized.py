"""The library's host code (argument checks, tuning, workspace layout, plan
bookkeeping) under AddressSanitizer and UndefinedBehaviorSanitizer: the HIP
source is rebuilt with both sanitizers on the host side only (the gfx950
device code is compiled as usual) into a temporary library, and the ABI
tests (tests/test_abi.py, which need no GPU) run again against it in a child
process with clang's sanitizer runtime preloaded.  Any memory error or
undefined behaviour they reach aborts the child."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_abi_under_host_sanitizers(tmp_path):
    runtimes = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not os.path.exists(HIPCC) or not runtimes:
        pytest.skip("hipcc or clang's sanitizer runtime not available")
    lib = tmp_path / "libpbspgemm_san.so"
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                           "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-Wno-unused-command-line-argument", *san,
                           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2002_11302_amd", "csrc"),
                           "-o", str(lib), os.path.join(ROOT, "paper_2002_11302_amd", "csrc", "pbspgemm.hip")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    env = dict(os.environ, LD_PRELOAD=runtimes[-1], PB_LIB=str(lib),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    log = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, log
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, log
    assert " passed" in r.stdout, log
