"""Host-side logic of bench.py (no GPU): algorithmic byte accounting, the
counter-summary reader and the one-GPU guard."""
import os
import subprocess
import sys

import bench
from synth.patterns import ISO, MONO, motif


class _G:
    n, m = 1000, 5000


def _stats(survivors, work, rows, counted_rows=0, counted_work=0, filter_rows=0,
           filter_entries=0):
    return {"survivors": survivors, "work": work, "rows": rows, "counted_rows": counted_rows,
            "counted_work": counted_work, "filter_rows": filter_rows,
            "filter_entries": filter_entries}


def test_kernel_bytes_follow_the_per_unit_figures():
    p = motif("cycle4")                       # k = 4: depths 2 (expand) and 3 (last level)
    st = _stats(survivors=70, work=[0, 0, 300, 900, 0], rows=[0, 0, 70, 40, 0],
                counted_rows=10, counted_work=200, filter_rows=50, filter_entries=600)
    out = bench.kernel_bytes([st], _G, [(p, ISO)])
    assert out["vertex_validator"] == bench.B_VERTEX * _G.n
    assert out["edge_scan"] == bench.B_ARC * _G.m + bench.B_ROW2 * 70
    assert out["expand"] == bench.B_CAND * 300 + 4 * 3 * 40
    assert out["last_level"] == bench.B_CAND * (900 - 200) + (4 * 3 + 24 + 4 * 3) * 10
    assert out["filter"] == (48 + 8 * 3) * 50 + 8 * 600
    assert out["index"] == 0
    st["index_arcs"] = 1200
    idx = bench.kernel_bytes([st], _G, [(p, MONO)])["index"]
    assert idx == 2 * (32 * _G.m + 8 * 1200 + 12 * (_G.n + 1))
    # a three-vertex pattern goes from depth 2 straight to the last level
    p3 = motif("cycle3")
    three = bench.kernel_bytes([_stats(5, [0, 0, 40, 0], [0, 0, 5, 0])], _G, [(p3, MONO)])
    assert three["expand"] == 0
    assert three["last_level"] == bench.B_CAND * 40


def test_measured_traffic_needs_a_summary_of_this_kernel_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "w_traffic.txt").write_text(
        "# header\n"
        "kernel=filter source_sha256=abc fetch_bytes_per_step=1000 write_bytes_per_step=400 "
        "dispatches_per_step=7\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "abc")
    assert bench.measured_traffic("w", "filter", 2) == 700      # (1000 + 400) / 2 launches
    assert bench.measured_traffic("w", "expand", 2) is None      # family not in the summary
    assert bench.measured_traffic("missing", "filter", 2) is None
    monkeypatch.setattr(bench, "kernel_source_sha", lambda: "other")
    assert bench.measured_traffic("w", "filter", 2) is None      # taken on other kernels


def test_committed_summaries_parse():
    for w in ("rmat20", "chunglu"):
        path = os.path.join(bench.ROOT, "profiles", f"{w}_traffic.txt")
        lines = [l for l in open(path) if l.startswith("kernel=")]
        assert lines, path
        for line in lines:
            fields = dict(kv.split("=", 1) for kv in line.split())
            assert {"source_sha256", "fetch_bytes_per_step", "write_bytes_per_step"} <= set(fields)
            assert float(fields["fetch_bytes_per_step"]) > 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def test_step_statistics():
    st = bench.step_statistics([0.010, 0.012, 0.011, 0.013, 0.009])
    assert st["median"] == 11.0 and st["min"] == 9.0 and st["max"] == 13.0 and st["n"] == 5
    assert abs(st["mean"] - 11.0) < 1e-9
    lo, hi = st["ci95"]
    # t(0.975, 4) = 2.776, s = 1.5811 ms, half width = 2.776 * 1.5811 / sqrt(5)
    assert abs((hi - lo) / 2 - 2.776445 * 1.581139 / 5 ** 0.5) < 1e-3
    assert "ci95" not in bench.step_statistics([0.5])
