"""The oracle's own pins, re-run on a build of the oracle instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer: an out-of-bounds access,
use after free, signed overflow or misaligned load anywhere in the C code
that the pins exercise aborts the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(os.environ.get("MDREF_LIB") is not None, reason="already the sanitizer run")
def test_oracle_pins_under_sanitizers():
    import oracle
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if asan is None or ubsan is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    lib = oracle.build(sanitize=True)
    env = dict(os.environ, MDREF_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    tests = sorted(os.path.join("tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f != "test_oracle_sanitized.py")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu",
                        "-p", "no:cacheprovider", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert "Sanitizer" not in r.stderr, tail
    assert r.returncode == 0, tail
    assert " passed" in r.stdout, tail
