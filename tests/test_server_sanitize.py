"""Sanitizer builds of the serving scheduler (host code only, no GPU).

tests/native/server_stress.cpp drives pp_server.cpp with a fake backend from
several threads under a budget that forces evictions; it is built with g++ and
run once under ThreadSanitizer and once under AddressSanitizer with
UndefinedBehaviorSanitizer.  Any report fails the run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "paper_2104_01636_amd", "csrc", "pp_server.cpp"),
       os.path.join(ROOT, "tests", "native", "server_stress.cpp")]


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_scheduler_under_sanitizer(san, tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "server_stress"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", f"-fsanitize={san}",
           "-fno-sanitize-recover=all", "-I" + os.path.join(ROOT, "include"), *SRC, "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=300)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "WARNING: ThreadSanitizer" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
    print(r.stdout)
