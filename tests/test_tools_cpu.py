"""Host-side helpers of the measurement path, on the CPU: the rocprofv3
summary tool (kernel names, the code hash that keys the traffic record, the
HBM traffic arithmetic on a synthetic counter database), the accuracy block
of the benchmark line, the benchmark's refusal of more than one GPU, and the
build entry point's reach of both build modules."""
import argparse
import json
import os
import sqlite3
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1609_05722_amd import rocprof_summary as rs  # noqa: E402


def test_short_name():
    assert rs.short_name("void fe::(anonymous namespace)::fused_step_kernel<7, "
                         "fe::(anonymous namespace)::MathF32<7, 3, false> >(fe::JobDesc const*, "
                         "int)") == "fused_step_kernel<7, MathF32<7, 3, false> >"
    mangled = ("_ZN2fe12_GLOBAL__N_117fused_step_kernelILi7ENS0_7MathP16ILi7ELi3EDF16bEEEEvPKNS0_"
               "7JobDescE")
    assert rs.short_name(mangled) == "fused_step_kernel<7, MathP16<7, 3, __bf16> >"
    assert rs.short_name(mangled.replace("DF16b", "DF16_")).endswith("_Float16> >")
    # with the waves-per-workgroup and mode template arguments
    mangled2 = ("_ZN2fe12_GLOBAL__N_117fused_step_kernelILi7ENS0_7MathP16ILi7ELi3EDF16bLi8EEELi2EEEv"
                "PKNS0_7JobDescE")
    assert rs.short_name(mangled2) == "fused_step_kernel<7, MathP16<7, 3, __bf16, 8>, 2>"


def test_code_hash_ignores_comments_only(tmp_path):
    a, b, c = tmp_path / "a.hip", tmp_path / "b.hip", tmp_path / "c.hip"
    a.write_text("int f(int x)\n{\n    return x + 1;  // one\n}\n")
    b.write_text("/* header */\nint f(int x) {\n  // note\n  return x + 1;\n}\n")
    c.write_text("int f(int x)\n{\n    return x + 2;\n}\n")
    assert rs.code_hash(str(a)) == rs.code_hash(str(b))
    assert rs.code_hash(str(a)) != rs.code_hash(str(c))


def _pmc_db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table pmc_events (dispatch_id int, name text, counter_name text, "
                "counter_value real)")
    for d, name, v in rows:
        # two instances per dispatch, summed by the tool
        con.execute("insert into pmc_events values (?, ?, ?, ?)", (d, name, counter, v / 2))
        con.execute("insert into pmc_events values (?, ?, ?, ?)", (d, name, counter, v / 2))
    con.commit()
    con.close()


def test_traffic_scales_by_the_copy(tmp_path):
    """FETCH reads half of a copy's bytes here, WRITE all of them: the step's
    counters are scaled by the same factors."""
    copy_bytes = 512 * 2 ** 20
    fdb, wdb = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    _pmc_db(fdb, "FETCH_SIZE", [(1, "copyBuffer", copy_bytes / 2 / 1024), (2, "copyBuffer", 4.0),
                                (3, "fused_step_kernel", 1000.0), (4, "fused_step_kernel", 1002.0)])
    _pmc_db(wdb, "WRITE_SIZE", [(1, "copyBuffer", copy_bytes / 1024),
                                (3, "fused_step_kernel", 500.0), (4, "fused_step_kernel", 500.0)])
    src = tmp_path / "k.hip"
    src.write_text("__global__ void k() {}\n")
    out = tmp_path / "t.json"
    rs.traffic(argparse.Namespace(fetch_db=fdb, write_db=wdb, kernel="fused_step",
                                  copy_kernel="copyBuffer", copy_bytes=float(copy_bytes),
                                  kernel_source=str(src), size=512, out=str(out)))
    rec = json.loads(out.read_text())
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["bytes_per_launch"] == pytest.approx(1001.0 * 1024 * 2 + 500.0 * 1024)
    assert rec["kernel_code_sha256_16"] == rs.code_hash(str(src))


def test_kernel_stats_by_launch_shape(tmp_path):
    """One kernel launched on two workloads: one line per launch shape with
    --by-grid, one merged line without."""
    db = str(tmp_path / "k.db")
    con = sqlite3.connect(db)
    con.execute("create table kernels (name text, duration real, grid_x int, grid_y int, "
                "grid_z int)")
    for d, g in ((100e3, 129024), (120e3, 129024), (30e3, 116736)):
        con.execute("insert into kernels values (?, ?, ?, 1, 1)", ("fused_step_kernel", d, g))
    con.commit()
    con.close()
    merged = rs.kernel_stats(db)
    assert len(merged) == 1 and merged[0]["calls"] == 3
    assert merged[0]["avg_us"] == pytest.approx(250.0 / 3)
    split = {r["grid"]: r for r in rs.kernel_stats(db, by_grid=True)}
    assert split[129024]["calls"] == 2 and split[129024]["avg_us"] == pytest.approx(110.0)
    assert split[116736]["avg_us"] == pytest.approx(30.0)


def test_accuracy_block():
    import bench
    g = np.random.default_rng(3)
    clean = g.uniform(0, 4, (32, 32))
    xo = clean + g.normal(0, 0.5, clean.shape)
    uo = 2 * np.sqrt(np.maximum(xo, 0) + 0.375)
    same = bench.accuracy({"fp32": (xo.copy(), uo.copy())}, uo, xo, clean, 4.0)
    assert same["fp32"]["max_abs_err_x"] == 0 and same["fp32"]["dpsnr_db"] == 0
    xg = xo.copy()
    xg[3, 4] += 0.25
    acc = bench.accuracy({"bf16": (xg, uo + 1e-3)}, uo, xo, clean, 4.0)["bf16"]
    assert acc["max_abs_err_x"] == pytest.approx(0.25, rel=1e-3)
    assert acc["rms_err_x"] == pytest.approx(0.25 / 32, rel=1e-2)
    assert acc["max_abs_err_u"] == pytest.approx(1e-3, rel=1e-3)
    p0 = 10 * np.log10(16 / np.mean((xo - clean) ** 2))
    p1 = 10 * np.log10(16 / np.mean((xg - clean) ** 2))
    assert acc["dpsnr_db"] == pytest.approx(p1 - p0, abs=1e-5)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_build_entry_resolves_both_build_modules():
    """build() reaches both build modules (not the oracle's re-exported
    function) and the oracle's build runs here."""
    import __graft_entry__ as g
    fe_build, oracle_build = g._builders()
    assert fe_build.__name__ == "paper_1609_05722_amd.build" and callable(fe_build.build)
    assert oracle_build.__name__ == "oracle.build" and callable(oracle_build.build)
    assert os.path.exists(oracle_build.build())
