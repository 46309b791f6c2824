"""The server's scheduler core (csrc/sched.hpp, HIP-free) with a fake
executor, built with g++ under ThreadSanitizer and AddressSanitizer: several
submitting threads, random device latencies, rounds that fail to launch, NaN
outputs, and shutdown with requests still pending (the core must finish them
and return)."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "sched_fake.cpp")


@pytest.mark.parametrize("san", ["thread", "address"])
def test_scheduler_core_under_sanitizer(tmp_path, san):
    exe = str(tmp_path / f"sched_{san}")
    cmd = ["g++", "-std=c++17", "-O1", "-g", f"-fsanitize={san}", "-fno-omit-frame-pointer", "-pthread",
           "-o", exe, SRC]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    # the environment may preload a library ahead of the sanitizer runtime
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:verify_asan_link_order=0"
    res = subprocess.run([exe], capture_output=True, text=True, timeout=240, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "OK" in res.stdout
    assert "WARNING: ThreadSanitizer" not in res.stderr, res.stderr
