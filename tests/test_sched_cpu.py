"""Builds and runs the host-only scheduler checks (tests/sched_test.cpp):
admission by memory budget in arrival order, per-tick counts, deferred
release, active cap.  No GPU involved."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_scheduler_host_logic(tmp_path):
    exe = tmp_path / "sched_test"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall",
                           "-fsanitize=address,undefined",
                           "-I" + os.path.join(ROOT, "paper_1609_05722_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sched_test.cpp"), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "OK"
