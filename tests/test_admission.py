"""The served form's admission policy on the CPU (no GPU): point-set
budget, submit checks, batches of one class in arrival order within the
scratch, request and work limits, cancellation, deadlines on a mock clock
and releasing point sets, against a fake allocator; built with
AddressSanitizer and UndefinedBehaviorSanitizer (host code only)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_admission_policy(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "admission_driver"
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-omit-frame-pointer", "-o", str(exe),
                           os.path.join(ROOT, "tests", "admission_driver.cpp")])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
