"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle.c is built with gcc -fsanitize=address,undefined (every report fatal)
into a temporary library, and tests/test_oracle.py runs against it in a
child interpreter with the ASan runtime preloaded.  A negative control reads
past the end of the position array through an out-of-range index and must be
stopped by ASan, which shows the sanitized library is the one loaded.
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "oracle.c")


def _runtime(name):
    if shutil.which("gcc") is None:
        return None
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    asan = _runtime("libasan.so")
    if asan is None or _runtime("libubsan.so") is None:
        pytest.skip("gcc sanitizer runtimes not installed")
    out = str(tmp_path_factory.mktemp("asan") / "liboracle_asan.so")
    subprocess.run(["gcc", "-O1", "-g", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                    "-fno-fast-math", "-ffp-contract=off", "-Wall",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-o", out, SRC, "-lm"], check=True)
    env = dict(os.environ)
    env.update(NBODY_ORACLE_LIB=out, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="4")
    return env


def test_oracle_pins_pass_under_asan_and_ubsan(sanitized):
    p = subprocess.run([sys.executable, "-m", "pytest", os.path.join(HERE, "test_oracle.py"),
                        "-q", "-x", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=sanitized, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stdout[-3000:] + p.stderr[-3000:]
    assert "passed" in p.stdout


def test_sanitizer_is_live(sanitized):
    code = ("import numpy as np, oracle\n"
            "x = np.zeros((16, 3)); v = np.zeros((16, 3)); m = np.ones(16)\n"
            "oracle.force(x, v, m, 0.1, np.array([16]))\n")
    p = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=sanitized,
                       capture_output=True, text=True, timeout=120)
    assert p.returncode != 0
    assert "AddressSanitizer" in p.stderr
