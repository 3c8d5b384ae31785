"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): oracle.c is rebuilt with -fsanitize=address,undefined and a
subset of the pin tests (1D rules, exact-rational brute force, invariants,
error norms, the matrix-based apply, the Hermite-like basis) runs against
that build in a child process.  Any out-of-bounds access, use after free or
undefined operation aborts the child with a report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["tests/test_oracle_1d.py", "tests/test_oracle_exact.py", "tests/test_oracle_invariants.py",
        "tests/test_oracle_errors.py", "tests/test_oracle_spmv.py", "tests/test_oracle_hermite.py"]


def test_pins_under_asan_and_ubsan():
    if os.environ.get("LD_PRELOAD"):
        pytest.skip("a library is preloaded already; AddressSanitizer's runtime has to come first")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime here")
    sys.path.insert(0, ROOT)
    from oracle import buildlib
    lib = buildlib.build_sanitized()
    env = dict(os.environ, DG_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "-k", "not convergence and not same_discrete_solution"] + PINS,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
