"""Host-side logic of bench.py, no GPU needed: the roofline arithmetic of the
expansion kernel, the guard that drops the measured HBM traffic once the
kernel source changes, and the single-GPU rule."""
import hashlib
import os
import subprocess
import sys
import types

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _level(ns, chunks, expanded, twins):
    return dict(ns_expand=ns, chunks=chunks, expanded=expanded, twins=twins)


def test_roofline_rows_only():
    # m = 64 int32: a child writes its 256-byte row + 32 bytes of records and
    # probe, so 1000 children in 288000 ns move 1 byte per ns = 1 GB/s
    system = types.SimpleNamespace(m=64)
    r = bench.roofline(system, [dict(level_stats=[_level(288000, 1, 1000, 0)])])
    assert r["achieved"] == 1.0
    assert r["bytes_per_launch"] == 288000
    assert r["avg_launch_us"] == 288.0
    assert r["frac"] == round(1.0 / 8000.0, 4)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0


def test_roofline_twins_and_steps():
    # two steps of two launches; 10 of the 1000 children of a step are twins
    # (12 bytes each): 990 x 288 + 10 x 12 = 285240 bytes per step
    system = types.SimpleNamespace(m=64)
    step = dict(level_stats=[_level(100000, 1, 400, 0), _level(185240, 1, 600, 10)])
    r = bench.roofline(system, [step, step])
    assert r["achieved"] == 1.0
    assert r["launches_per_step"] == 2
    assert r["bytes_per_launch"] == 285240 // 2
    assert r["expand_us_per_step"] == 285.24


def test_traffic_guard(tmp_path, monkeypatch):
    src = tmp_path / "kernels.hip"
    src.write_text("// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "traffic.md"
    prof.write_text(f"# counters\n\n- `traffic_bytes_per_launch`: `12345`\n- `kernel_source_sha256`: `{sha}`\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(prof))
    assert bench.measured_traffic() == 12345
    src.write_text("// kernel source, changed\n")
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic() is None


def test_committed_traffic_file_parses():
    # the committed counter summary carries both fields the guard reads
    text = open(bench.TRAFFIC_FILE).read()
    assert "- `traffic_bytes_per_launch`: `" in text and "- `kernel_source_sha256`: `" in text


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "--gpus must be 1" in res.stderr
    assert res.stdout == ""
