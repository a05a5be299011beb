"""Host-side logic of bench.py, no GPU needed: the roofline arithmetic of the
dominant kernels, the batched workload's critical-path bound, and the
single-GPU rule."""
import os
import subprocess
import sys
import types

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _level(ns, chunks, expanded=0, twins=0, new=0, mfma=0):
    return dict(ns_expand=ns, chunks=chunks, expanded=expanded, twins=twins, new_configs=new, mfma_ops=mfma)


def test_roofline_new_rows():
    # 1000 new rows of 2064 bytes (2 KiB row + 16 B entry) in 2064000 ns: 1 GB/s
    r = bench.hbm_roofline([dict(level_stats=[_level(1032000, 1, new=500), _level(1032000, 1, new=500)])],
                           "k", 2064, 2048)
    assert r["roofline"]["achieved"] == 1.0
    assert r["roofline"]["frac"] == round(1.0 / 8000.0, 4)
    assert r["roofline"]["bound"] == "hbm" and r["roofline"]["unit"] == "GB/s" and r["roofline"]["peak"] == 8000.0
    assert r["dominant_kernel"]["bytes_per_launch"] == 1032000
    assert r["dominant_kernel"]["avg_launch_us"] == 1032.0
    assert r["dominant_kernel"]["launches_per_step"] == 2


def test_roofline_lane_form_per_child_and_steps():
    # two steps of two launches; each of the 1000 children computed in a step
    # writes a 256-byte row + 32 bytes (twins are never computed, so the
    # level's twin count adds nothing): 288000 bytes per step
    step = dict(level_stats=[_level(100000, 1, 400, 0), _level(188000, 1, 600, 10)])
    r = bench.hbm_roofline([step, step], "k_expand_lane", None, 256, per_child=True)
    assert r["roofline"]["achieved"] == 1.0
    assert r["dominant_kernel"]["launches_per_step"] == 2
    assert r["dominant_kernel"]["bytes_per_launch"] == 288000 // 2
    assert r["dominant_kernel"]["kernel_us_per_step"] == 288.0


def test_mfma_utilisation():
    # 5e12 ops in 1e6 ns = 5e15 op/s: the whole int8 peak
    r = bench.mfma_util([dict(level_stats=[_level(10 ** 6, 1, mfma=5 * 10 ** 12)])])
    assert r["achieved_tops"] == 5000.0 and r["frac"] == 1.0


def test_batch_work_per_step():
    systems = [types.SimpleNamespace(r=5, n_syn=4, m=3), types.SimpleNamespace(r=128, n_syn=256, m=64)]
    assert bench.batch_work(systems) == [12, 448]


def test_batch_bound_terms():
    """Clock 2.4 GHz: one CU does 64 integer operations and 32 LDS words per
    clock, the chip 256 times the former.  System a: r 1, 767 synapses, m 1
    (work 769 per step); b: r 1, 7 synapses, m 4088 (work 4096, 7 gathers)."""
    a = types.SimpleNamespace(r=1, n_syn=767, m=1)
    b = types.SimpleNamespace(r=1, n_syn=7, m=4088)
    steps = [2400, 2400]
    bound, chip, valu, lds, work = bench.batch_bound([a, b], steps)
    assert work.tolist() == [769 * 2400, 4096 * 2400]
    # b's work at 64 per clock: 4096 * 2400 / 64 clocks = 153600 clocks = 64 us
    assert abs(valu - 64e-6) < 1e-12
    # a's gathers at 32 per clock: 767 * 2400 / 32 = 57525 clocks = 23.97 us
    assert abs(lds - 767 * 2400 / 32 / 2.4e9) < 1e-15
    # both systems at 256 CUs x 64 per clock
    assert abs(chip - (769 + 4096) * 2400 / (256 * 64 * 2.4e9)) < 1e-15
    assert bound == valu
    # with a's synapses multiplied the LDS term takes over
    a.n_syn = 7670
    a.r = 1
    bound, chip, valu, lds, _ = bench.batch_bound([a, b], steps)
    assert bound == lds and abs(lds - 7670 * 2400 / 32 / 2.4e9) < 1e-15


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "--gpus must be 1" in res.stderr
    assert res.stdout == ""
