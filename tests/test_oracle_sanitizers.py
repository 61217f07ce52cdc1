"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's C++ source is built with -fsanitize=address,undefined (every finding fatal) and
the CPU pins of the oracle run against that build in a child process with the ASan runtime
preloaded: an out-of-bounds access, use after free, signed overflow, misaligned access or
invalid shift anywhere those pins reach fails this test.  Leak checking is off (the Python
interpreter keeps allocations alive until exit).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PINS = ["test_oracle_atoms.py", "test_oracle_consistency.py", "test_oracle_coupling.py",
        "test_oracle_d3q27.py", "test_oracle_gradient.py", "test_oracle_lattice.py",
        "test_oracle_noise.py", "test_oracle_trt.py"]


def _runtime(name):
    out = subprocess.run(["g++", "-print-file-name=" + name], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if out.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    from oracle import oracle as O
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("the compiler's AddressSanitizer runtime is not installed")
    lib = O.build_sanitized(str(tmp_path / "liblbmd_oracle_asan.so"))
    env = dict(os.environ)
    pre = env.get("LD_PRELOAD")
    env["LD_PRELOAD"] = asan + (":" + pre if pre else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["LBMD_ORACLE_LIB"] = lib
    env["OMP_NUM_THREADS"] = env.get("OMP_NUM_THREADS", "4")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
           *[os.path.join(ROOT, "tests", f) for f in PINS]]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    print(tail)
    assert r.returncode == 0, tail
    assert "passed" in r.stdout
