"""Builds and runs the host-only planner checks (tests/plan_test.cpp)
against libfe.so: tile grids, tile heights within each variant's LDS limit,
tuning candidates, batch signatures.  No GPU involved."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1609_05722_amd")


def test_planner_host_logic(tmp_path):
    lib = os.path.join(PKG, "libfe.so")
    if not os.path.exists(lib):
        pytest.skip("libfe.so not built")
    exe = tmp_path / "plan_test"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-D__HIP_PLATFORM_AMD__",
                           "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"),
                           "-I" + os.path.join(PKG, "csrc"),
                           os.path.join(ROOT, "tests", "plan_test.cpp"), lib,
                           "-Wl,-rpath," + PKG, "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "OK"
