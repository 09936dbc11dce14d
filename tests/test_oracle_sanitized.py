"""The oracle's pins again, with the oracle built under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): an out-of-bounds access, a use after
free, a signed overflow or a misaligned load anywhere in the oracle's C code on
the pins' inputs aborts the run."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _asan_runtime():
    try:
        out = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True, check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.timeout(900)
def test_oracle_pins_under_asan_ubsan():
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc's ASan runtime is not installed")
    env = dict(os.environ)
    env.update({
        "RBF_ORACLE_SANITIZE": "1",
        "LD_PRELOAD": rt,
        # Python's own allocations are not the oracle's: leaks are not checked
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "OMP_NUM_THREADS": "4",
    })
    sys.path.insert(0, ROOT)
    build = subprocess.run([sys.executable, "-c", "import oracle; oracle.build()"], cwd=ROOT,
                           env={k: v for k, v in env.items() if k != "LD_PRELOAD"},
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-4000:]
    run = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                          os.path.join(HERE, "test_oracle_pins.py")],
                         cwd=ROOT, env=env, capture_output=True, text=True)
    tail = (run.stdout[-3000:] + "\n" + run.stderr[-6000:])
    assert run.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in run.stderr, tail
    assert "runtime error:" not in run.stderr, tail
