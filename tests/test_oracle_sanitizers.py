"""The oracle's pins again on an AddressSanitizer + UndefinedBehaviorSanitizer
build of the oracle (host code; no GPU): out-of-bounds or use-after-free
accesses, signed overflow, misaligned or null accesses abort the run.

The instrumented library is loaded into a fresh Python process that preloads
the sanitizer runtime (the interpreter itself is not instrumented; its
leaks are not checked)."""
import os
import subprocess
import sys

import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime():
    p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if p.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan():
    asan = _runtime()
    if asan is None:
        pytest.skip("gcc has no AddressSanitizer runtime here")
    O.build(sanitize=True)
    env = dict(os.environ)
    env.update(ADG_ORACLE_SANITIZED="1", LD_PRELOAD=asan, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    files = ["tests/test_oracle_pins.py", "tests/test_oracle_adjoint.py", "tests/test_oracle_boundaries.py",
             "tests/test_oracle_limiter.py", "tests/test_linear_form.py"]
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu and not slow", "-p",
                        "no:cacheprovider"] + files, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=1800)
    tail = (p.stdout + p.stderr)[-3000:]
    assert p.returncode == 0, tail
    assert "AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, tail
