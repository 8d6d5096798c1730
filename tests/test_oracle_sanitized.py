"""The oracle's C code built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, OpenMP on, four threads) and run by tests/sanitize_oracle.c through
every entry point of the three-way and N-way oracles: no memory error, leak
or undefined behaviour."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    exe = tmp_path / "sanitize_oracle"
    srcs = [os.path.join(HERE, "sanitize_oracle.c"), os.path.join(ROOT, "oracle", "sacd_oracle.c"),
            os.path.join(ROOT, "oracle", "sacd_oracle_n.c")]
    cmd = [gcc, "-std=c11", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-o", str(exe)] + srcs + ["-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower() and "cannot find" in r.stderr.lower():
        pytest.skip("no sanitizer runtime: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, OMP_NUM_THREADS="4", ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    if "does not come first in initial library list" in r.stderr:
        pytest.skip("another library is preloaded ahead of the sanitizer runtime")
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "sanitized oracle run ok" in r.stdout
