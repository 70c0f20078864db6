"""The host set-up code (csrc/host_tables.hpp) built for the CPU with
AddressSanitizer and UndefinedBehaviorSanitizer and run on several box shapes
(tests/host_tables_check.cpp): no sanitizer report, and the tables it builds
(geometry, Gauss-Jordan inverse, Vanka local inverses, dense coarsest
inverse, V1 colour lists) check out against the stencil of Eq. 2."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_tables_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "host_tables_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(HERE, "host_tables_check.cpp"), "-o", str(exe)]
    build = subprocess.run(cmd, capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0 and run.stdout.strip() == "ok", run.stdout + run.stderr
