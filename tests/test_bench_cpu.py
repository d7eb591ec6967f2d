"""The benchmark's bookkeeping, without a GPU: the one-GPU guard, the
algorithmic byte count, and the rocprofv3 summaries behind the roofline
(counter calibration, the kernel digest that keys the traffic figure)."""
import json
import os
import sqlite3
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_counts_every_event_once():
    stats = {"global_relabels": 3, "bfs_vertices": 10, "bfs_arcs": 100, "pr_vertex_cycles": 7,
             "pr_arcs": 50, "pushes": 4, "relabels": 2, "rie_arcs": 9, "rie_saturations": 1,
             "updates": 5, "clamps": 2, "source_pushes": 6, "rounds": 99, "call_ms": 1.5}
    n = 1000
    want = 3 * n * bench.BYTES["height_reset_vertex"]
    want += sum(stats[k] * v for k, v in bench.BYTES.items() if k in stats)
    assert bench.algorithmic_bytes(stats, n) == want
    # counters the model does not price (rounds, times) add nothing
    assert bench.algorithmic_bytes({"global_relabels": 0, "rounds": 5}, n) == 0


def _pmc_db(path, counter, calib_kib, loop_kib):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (kernel_name text, dispatch_id int, counter_name text, value real)")
    rows = [("void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel>", i, counter, v)
            for i, v in enumerate(calib_kib)]
    rows += [("void mf::k_loop<1024, 4>(mf::DevGraph, mf::LoopParams)", 10 + i, counter, v)
             for i, v in enumerate(loop_kib)]
    rows += [("mf::k_clamp(mf::DevGraph, long const*, long)", 50, counter, 123.0)]
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_pmc_summary_scales_by_the_calibration_and_keys_by_the_kernel(tmp_path, monkeypatch, capsys):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "abc123")
    # FETCH_SIZE reads half the bytes of a known 256 MiB copy (factor 2), WRITE_SIZE all of them
    _pmc_db(tmp_path / "f.db", "FETCH_SIZE", [131072, 131072, 131072], [999.0, 999.0, 100.0, 300.0])
    _pmc_db(tmp_path / "w.db", "WRITE_SIZE", [262144], [7.0, 7.0, 40.0, 60.0])
    bench.summarize_pmc(str(tmp_path / "f.db"), str(tmp_path / "w.db"), "grid512", 256, 2, "cmd")
    rec = json.load(open(tmp_path / "profiles" / "k_loop_grid512_pmc.json"))
    assert rec["kernel_digest"] == "abc123" and rec["command"] == "cmd"
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    assert rec["fetch_launches"] == 2 and rec["write_launches"] == 2  # the first two left out
    assert rec["fetch_bytes_per_launch"] == pytest.approx(200.0 * 1024 * 2.0)
    assert rec["write_bytes_per_launch"] == pytest.approx(50.0 * 1024)
    assert rec["bytes_per_launch"] == pytest.approx(200.0 * 2048 + 50.0 * 1024)
    assert "HBM bytes per k_loop launch" in capsys.readouterr().out
    # the traffic figure is reported only while the kernel sources are unchanged
    assert bench.load_traffic("grid512", "bytes_per_launch") == pytest.approx(rec["bytes_per_launch"])
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "changed")
    assert bench.load_traffic("grid512", "bytes_per_launch") is None
    assert bench.load_traffic("rmat20", "bytes_per_launch") is None  # no summary for it here


def test_pmc_summary_refuses_a_run_without_the_calibration(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "abc123")
    _pmc_db(tmp_path / "f.db", "FETCH_SIZE", [], [1.0, 2.0, 3.0])
    _pmc_db(tmp_path / "w.db", "WRITE_SIZE", [262144], [1.0, 2.0, 3.0])
    with pytest.raises(SystemExit):
        bench.summarize_pmc(str(tmp_path / "f.db"), str(tmp_path / "w.db"), "grid512", 256, 2, "cmd")


def test_kernel_trace_summary_table(tmp_path, capsys):
    con = sqlite3.connect(tmp_path / "k.db")
    con.execute("create table kernels (name text, duration int)")
    con.executemany("insert into kernels values (?, ?)",
                    [("k_loop", 2_000_000), ("k_loop", 4_000_000), ("k_clamp", 1_000_000)])
    con.commit()
    con.close()
    bench.summarize_profile(str(tmp_path / "k.db"))
    out = capsys.readouterr().out.splitlines()
    assert out[0].startswith("| kernel | calls")
    row = [c.strip() for c in out[2].split("|")]
    assert row[1] == "`k_loop`" and row[2] == "2" and row[3] == "6.000" and row[4] == "3.0000"
    assert float(row[7]) == pytest.approx(100.0 * 6 / 7, abs=0.01)
