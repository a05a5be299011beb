"""Benchmark: new configurations per second of the breadth-first expansion.

One step is one complete breadth-first walk of the dense int8 workload (seeded
synthetic system, m = 512 neurons, 3 rules per neuron, E = a^i (a^j)* with
i in [1,4], j in [0,3], p in [0,4] so that M_Pi's entries lie in [-4, 4],
out-degree 64, C0 uniform in [0, 4], int32 counts, seed 0) from C0 to depth 3
with every level truncated to its first 1e6 new configurations: every level
runs applicability + Psi, the prefix sums, the expansion C' = C + S.M on the
int8 matrix cores, the visited-set insert and the ordered commit, all on the
GPU through the C ABI.  The value is new (deduplicated) configurations per
second over the timed steps; inputs are resident in HBM before timing.

The JSON line also carries the roofline of the dominant kernel (device time
from HIP events the library records on its stream just before and after each
launch of it, inside the timed region), its int8 matrix-core utilisation, the
same walk on the plain sparse form (the speedup the metric names), the CPU
oracle timed on a bounded sample of the same workload, and secondary lines
for the plain-sparse, batched and large workloads, each with its own roofline
and CPU baseline, and one for the plain-sparse system with rule delays.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "new configurations/sec (deduped) per BFS step; int8-MFMA/batched vs plain sparse"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
INT8_PEAK_TOPS = 5000.0      # MI355X dense int8 matrix cores, published (no sparsity)
# Vector ALU for 32-bit integer work: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz =
# 39.3e12 operations per second (the published fp32 157.3 TFLOP/s counts an FMA as
# 2 flops and two fp32 values per packed instruction; 32-bit integer adds and
# compares are not packed)
CLOCK_GHZ = 2.4
INT_VALU_PER_CU = 64
VALU_PEAK_GOPS = 256 * INT_VALU_PER_CU * CLOCK_GHZ
CU_PEAK_GOPS = INT_VALU_PER_CU * CLOCK_GHZ
# LDS: 32 banks of 4 bytes per clock per CU, so a gather of 32-bit words from
# LDS takes at least one clock per 32 words
LDS_WORDS_PER_CU = 32
ENTRY_BYTES = 16             # visited-set entry written per new configuration
# bytes per child of the one-neuron-per-lane expansion besides its row: key 8,
# parent 4, child index 8, probe slot 4, visited-set entry 8
LANE_CHILD_EXTRA = 32
# bytes per child of the sparse (pull) expansion besides its row: key 8, parent 4, child index 8
SPARSE_CHILD_EXTRA = 20

DENSE_WORKLOAD = ("dense_int8: seeded SN P system m=512, 3 rules/neuron (r=1536), E=a^i(a^j)* i in [1,4] "
                  "j in [0,3], p in [0,4] (M entries in [-4,4], int8), out-degree 64, C0 in [0,4], int32 "
                  "counts; BFS depth 3, frontier_cap 1e6 per level, chunks of 2^20 children (seed 0)")
PLAIN_WORKLOAD = ("plain_sparse: m=64, 2 rules/neuron (r=128), i in [1,4] j in [0,3] p in {0,1}, out-degree 4, "
                  "C0 in [0,4], int32; BFS until a level reaches 1e5 configurations (seed 0)")
LARGE_WORKLOAD = ("large: m=4096, 4 rules/neuron (r=16384), out-degree 16, C0 in [0,8], uint16; BFS depth 3, "
                  "frontier_cap 4e6 per level, chunks of 2^22 children (seed 0)")
DELAY_WORKLOAD = ("plain_sparse_delays: the plain_sparse system (m=64, seed 0) with rule delays: each rule gets "
                  "one with probability 1/2, uniform in [1,3] (delay stream seed 0; 45 of 64 neurons delayed), "
                  "rows of counts plus (wait, pend) per delayed neuron, int32; BFS until a level reaches 1e5 "
                  "configurations")
BATCH_WORKLOAD = ("batched_uneven: 256 systems, m in [16,1024], 1-3 rules and out-degree 2-32 per neuron, "
                  "10k deterministic steps each, one graph-replayed launch (seeds 0-255)")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    model = platform.processor() or ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(nproc=os.cpu_count(), cpu_model=model)


def device_rows(system, rows):
    import numpy as np
    import torch

    a = np.asarray(rows, dtype=np.int64)
    a = a.astype(np.uint16).view(np.int16) if system.count_type == "u16" else a.astype(np.int32)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


class Walk:
    """A loaded handle plus its device buffers, for timed snp_run calls."""

    def __init__(self, system, path, cap, depth, stop, chunk, out_cap, profile, tune=False, cache=None):
        import numpy as np
        import torch

        from paper_1104_1824_amd import snp

        self.snp, self.system, self.depth, self.out_cap = snp, system, depth, out_cap
        self.h = snp.snp_load(system, path=path, frontier_cap=cap, stop_at_cap=stop, max_rows=out_cap, chunk=chunk,
                              profile=profile)
        # rows may carry more entries than the m counts (delay states): width from the library
        c0 = np.asarray(system.c0, dtype=np.int64)
        self.c0 = device_rows(system, np.concatenate([c0, np.zeros(self.h.m - c0.shape[0], dtype=np.int64)]))
        dt = torch.int16 if system.count_type == "u16" else torch.int32
        self.out = torch.empty((out_cap, self.h.m), dtype=dt, device="cuda")
        # launch settings timed on this very walk, before (and outside) the timed region;
        # with a cache file, settings found there are used as they are
        self.tuning = None
        if tune and cache and snp.snp_load_tuning(self.h, cache, depth):
            self.tuning = dict(snp.snp_get_tuning(self.h), cached=True)
        elif tune:
            self.tuning = snp.snp_autotune(self.h, self.c0, depth, self.out, out_cap, cache)

    def run(self):
        return self.snp.snp_run(self.h, self.c0, self.depth, self.out, self.out_cap)

    def timed(self, steps, warmup):
        import torch

        for _ in range(warmup):
            self.run()
        torch.cuda.synchronize()
        results = []
        t0 = time.perf_counter()
        for _ in range(steps):
            results.append(self.run())
        torch.cuda.synchronize()
        return results, time.perf_counter() - t0

    def close(self):
        self.h.close()
        del self.out


def totals(results, key):
    return sum(st[key] for r in results for st in r["level_stats"])


# Source files of each measured kernel: the traffic a profiles/*_traffic.md
# summary records is reported only while their SHA-256 is the one it names.
KERNEL_SOURCES = {
    "k_expand_int8": ["paper_1104_1824_amd/csrc/snp_int8.hip", "paper_1104_1824_amd/csrc/snp_device.hpp",
                      "paper_1104_1824_amd/csrc/snp_internal.hpp"],
    "k_expand_lane": ["paper_1104_1824_amd/csrc/snp_kernels.hip", "paper_1104_1824_amd/csrc/snp_device.hpp",
                      "paper_1104_1824_amd/csrc/snp_internal.hpp"],
    "k_expand_sparse": ["paper_1104_1824_amd/csrc/snp_kernels.hip", "paper_1104_1824_amd/csrc/snp_device.hpp",
                        "paper_1104_1824_amd/csrc/snp_internal.hpp"],
}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter
    summaries (profiles/*_traffic.md), or None when none matches the current
    kernel sources."""
    import glob
    import hashlib
    import re

    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, []):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    want = h.hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        fields = dict(re.findall(r"^- `(\w+)`: `([^`]*)`", open(path).read(), re.M))
        if fields.get("kernel") == kernel and fields.get("workload") == workload:
            if fields.get("kernel_source_sha256") == want:
                return int(fields["traffic_bytes_per_launch"])
    return None


def hbm_roofline(results, kernel, bytes_per_new, rb, per_child=False, workload=None, child_extra=LANE_CHILD_EXTRA):
    """Roofline of the expansion kernel: algorithmic bytes over its device time
    (HIP events around each launch).  Algorithmic bytes = every new configuration's
    row plus its visited-set entry (bytes_per_new); with per_child, the
    expansion's own per-child bytes instead (the row of every child computed,
    plus its records: child_extra bytes)."""
    ns = totals(results, "ns_expand")
    launches = totals(results, "chunks")
    if per_child:
        moved = totals(results, "expanded") * (rb + child_extra)
    else:
        moved = totals(results, "new_configs") * bytes_per_new
    achieved = moved / max(1, ns)  # bytes per ns = GB/s
    steps = max(1, len(results))
    return dict(
        roofline=dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS, unit="GB/s",
                      frac=round(achieved / HBM_PEAK_GBS, 4),
                      traffic=measured_traffic(kernel, workload) if workload else None),
        dominant_kernel=dict(kernel=kernel, launches_per_step=launches // steps,
                             bytes_per_launch=round(moved / max(1, launches)),
                             avg_launch_us=round(ns / max(1, launches) / 1e3, 3),
                             kernel_us_per_step=round(ns / 1e3 / steps, 2)),
    )


def mfma_util(results):
    ops = totals(results, "mfma_ops")
    ns = totals(results, "ns_expand")
    tops = ops / max(1, ns) / 1e3  # ops per ns = Gop/s; / 1e3 = Top/s
    return dict(ops_per_step=ops // max(1, len(results)), achieved_tops=round(tops, 3), peak_tops=INT8_PEAK_TOPS,
                frac=round(tops / INT8_PEAK_TOPS, 6))


# ---------------------------------------------------------------------------
# headline: the dense workload on the int8 matrix cores
# ---------------------------------------------------------------------------
def dense_system():
    import synth

    return synth.config_system(3, 0)


def run_dense(steps, warmup, tune, cache=None):
    from paper_1104_1824_amd import snp

    s = dense_system()
    log(f"dense m=512 seed 0, int8 path: warmup {warmup}, steps {steps}")
    w = Walk(s, snp.SNP_PATH_INT8, 1000000, 3, False, 1 << 20, 3000001, profile=1, tune=tune, cache=cache)
    if w.tuning:
        log(f"tuned launch settings: {w.tuning}")
    results, dt = w.timed(steps, warmup)
    w.close()
    results[-1]["tuning"] = w.tuning
    new = results[-1]["n_configs"] - 1
    assert all(r["n_configs"] - 1 == new for r in results)
    log(f"levels {results[-1]['level_sizes'].tolist()}, {new} new per walk, {dt / steps * 1e3:.3f} ms/walk")
    return s, results, dt


def run_dense_sparse(reps=1, tune=True):
    from paper_1104_1824_amd import snp

    log("dense m=512 seed 0, plain sparse path (the speedup's reference)")
    w = Walk(dense_system(), snp.SNP_PATH_SPARSE, 1000000, 3, False, 1 << 20, 3000001, profile=1, tune=tune)
    results, dt = w.timed(reps, 1)
    w.close()
    return dict(ms_per_walk=round(dt / reps * 1e3, 3), new_configs=int(results[-1]["n_configs"] - 1),
                configs_per_s=round((results[-1]["n_configs"] - 1) * reps / dt, 1), tuning=w.tuning)


def cpu_dense(budget_s=10.0):
    """The oracle on level 1 of the dense workload, capped at 1e5 new
    configurations (about 3e5 children enumerated), repeated for budget_s."""
    import oracle

    oracle.build(force=False)
    s = dense_system()
    n_new, runs = 0, 0
    t0 = time.perf_counter()
    while True:
        res = oracle.bfs(s, max_depth=1, frontier_cap=100000, rows_cap=100001)
        n_new += int(res.level_sizes[1:].sum())
        runs += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=round(n_new / dt, 1), unit="configs/s", cores=1, kind="oracle",
                sample=f"{runs} x level 1 of the same workload capped at 1e5 new configurations (seed 0), "
                       f"single-threaded C oracle, {dt:.1f} s", host=host_info())


# ---------------------------------------------------------------------------
# secondary: plain sparse, batched, large
# ---------------------------------------------------------------------------
def cpu_plain(budget_s=5.0):
    import oracle
    import synth

    oracle.build(force=False)
    s = synth.config_system(2, 0)
    n_new, runs, t0 = 0, 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        res = oracle.bfs(s, max_depth=1000, frontier_cap=100000, stop_at_cap=True, rows_cap=1 << 18)
        n_new += int(res.level_sizes[1:].sum())
        runs += 1
    dt = time.perf_counter() - t0
    return dict(value=round(n_new / dt, 1), unit="configs/s", cores=1, kind="oracle",
                sample=f"{runs} complete walks of the same workload, single-threaded, {dt:.1f} s")


def cpu_large():
    import oracle
    import synth

    oracle.build(force=False)
    s = synth.config_system(5, 0)
    t0 = time.perf_counter()
    res = oracle.bfs(s, max_depth=1, frontier_cap=2000, rows_cap=2001)
    dt = time.perf_counter() - t0
    return dict(value=round(int(res.level_sizes[1:].sum()) / dt, 1), unit="configs/s", cores=1, kind="oracle",
                sample=f"level 1 of the same workload capped at 2000 new configurations "
                       f"({int(res.enumerated[0])} children enumerated), single-threaded, {dt:.1f} s")


def plain_line(steps=50, warmup=5, cpu=None, tune=True, cache=None):
    import synth
    from paper_1104_1824_amd import snp

    s = synth.config_system(2, 0)
    log("plain sparse m=64 seed 0, sparse path")
    w = Walk(s, snp.SNP_PATH_SPARSE, 100000, 1000, True, 1 << 17, 200000, profile=1, tune=tune, cache=cache)
    results, dt = w.timed(steps, warmup)
    w.close()
    new = results[-1]["n_configs"] - 1
    line = dict(workload=PLAIN_WORKLOAD, value=round(steps * new / dt, 1), unit="configs/s",
                ms_per_step=round(dt / steps * 1e3, 4), levels=results[-1]["level_sizes"].tolist(), dtype="int32",
                tuning=w.tuning)
    line.update(hbm_roofline(results, "k_expand_lane", None, s.m * 4, per_child=True, workload="plain_sparse"))
    line["cpu_baseline"] = cpu
    return line


def delay_system():
    import synth
    from synth.systems import with_delays

    return with_delays(synth.config_system(2, 0), 0, d_max=3)


def cpu_delays(budget_s=5.0):
    import oracle

    oracle.build(force=False)
    s = delay_system()
    n_new, runs, t0 = 0, 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        res = oracle.bfs(s, max_depth=1000, frontier_cap=100000, stop_at_cap=True, rows_cap=1 << 19)
        n_new += int(res.level_sizes[1:].sum())
        runs += 1
    dt = time.perf_counter() - t0
    return dict(value=round(n_new / dt, 1), unit="configs/s", cores=1, kind="oracle",
                sample=f"{runs} complete walks of the same workload, single-threaded, {dt:.1f} s")


def delays_line(steps=20, warmup=3, cpu=None, tune=True, cache=None):
    from paper_1104_1824_amd import snp

    s = delay_system()
    log("plain sparse m=64 seed 0 with delays, sparse path")
    w = Walk(s, snp.SNP_PATH_SPARSE, 100000, 1000, True, 1 << 17, 400000, profile=1, tune=tune, cache=cache)
    rb = w.h.m * 4
    results, dt = w.timed(steps, warmup)
    w.close()
    new = results[-1]["n_configs"] - 1
    line = dict(workload=DELAY_WORKLOAD, value=round(steps * new / dt, 1), unit="configs/s",
                ms_per_step=round(dt / steps * 1e3, 4), levels=results[-1]["level_sizes"].tolist(), dtype="int32",
                row_entries=rb // 4, tuning=w.tuning)
    line.update(hbm_roofline(results, "k_expand_sparse", None, rb, per_child=True, workload="delays",
                             child_extra=SPARSE_CHILD_EXTRA))
    line["cpu_baseline"] = cpu
    return line


def batch_work(systems):
    """Algorithmic integer operations per step of every system: one
    applicability test per rule, one gather per synapse, one update per neuron."""
    return [s.r + s.n_syn + s.m for s in systems]


def batch_bound(systems, steps_done):
    """Times (s) a batched launch cannot beat, from unit counts: the batch's
    work at the chip's 32-bit vector rate, each system's work at one CU's
    vector rate, and each system's in-synapse gathers at one CU's LDS rate.
    Returns (bound, chip, largest CU vector term, largest CU LDS term, work)."""
    import numpy as np

    done = np.asarray(steps_done, dtype=np.int64)
    work = np.asarray(batch_work(systems), dtype=np.int64) * done
    gathers = np.asarray([s.n_syn for s in systems], dtype=np.int64) * done
    t_chip = work.sum() / (VALU_PEAK_GOPS * 1e9)
    t_valu = work / (CU_PEAK_GOPS * 1e9)
    t_lds = gathers / (LDS_WORDS_PER_CU * CLOCK_GHZ * 1e9)
    bound = max(t_chip, float(np.maximum(t_valu, t_lds).max()))
    return bound, t_chip, float(t_valu.max()), float(t_lds.max()), work


def batched_line(reps=3, cpu=None, largest=False):
    """The batched launch; largest=True runs only the workload's largest
    system (the one that bounds the launch), for per-step counters."""
    import numpy as np
    import torch

    import synth
    from paper_1104_1824_amd import snp

    systems = synth.batched_systems(0, 256)
    if largest:
        systems = [max(systems, key=lambda x: x.m)]
        log(f"batched deterministic launch, the largest system alone (m={systems[0].m}) x 10k steps")
    else:
        log("batched deterministic launch, 256 systems x 10k steps")
    b = snp.snp_batch_load(systems)
    off = snp.snp_batch_offsets(b)
    c0 = torch.from_numpy(np.concatenate([x.c0 for x in systems]).astype(np.int32)).cuda()
    fin = torch.empty(int(off[-1]), dtype=torch.int32, device="cuda")
    res = snp.snp_batch_run(b, c0, 10000, fin)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = snp.snp_batch_run(b, c0, 10000, fin)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    shape = snp.snp_batch_shape(b)
    b.close()
    done = res["steps_done"].astype(np.int64)
    steps_total = int(done.sum())
    t_min, t_chip, t_valu, t_lds, work = batch_bound(systems, done)
    line = dict(workload=BATCH_WORKLOAD + (", largest system alone" if largest else ""),
                value=round(steps_total / dt, 1), unit="system-steps/s",
                ms_per_launch=round(dt * 1e3, 3), dtype="int32", threads_per_system=shape[0],
                neurons_per_thread=shape[1],
                roofline=dict(bound="alu", achieved=round(work.sum() / dt / 1e9, 2),
                              peak=round(work.sum() / t_min / 1e9, 2), unit="Gop/s",
                              frac=round(t_min / dt, 4), traffic=None,
                              critical_path_ms=round(t_min * 1e3, 3),
                              chip_valu_ms=round(t_chip * 1e3, 3), cu_valu_ms=round(t_valu * 1e3, 3),
                              cu_lds_ms=round(t_lds * 1e3, 3),
                              largest_system_ops=int(work.max()), total_ops=int(work.sum())),
                cpu_baseline=cpu)
    return line


def _det(seed):
    import oracle
    import synth

    return oracle.deterministic(synth.batched_systems(seed, 1)[0], 10000).steps_done


def cpu_batched(sample=16):
    """The oracle's single-branch runs: the first `sample` systems on one core,
    and all 256 on a pool of forked processes (one system per task).  Run
    before this process touches the GPU."""
    import multiprocessing

    import oracle
    import synth

    oracle.build(force=False)
    systems = synth.batched_systems(0, 256)
    log(f"batched: CPU oracle, {sample} systems on one core")
    t0 = time.perf_counter()
    steps1 = sum(oracle.deterministic(s, 10000).steps_done for s in systems[:sample])
    dt1 = time.perf_counter() - t0
    workers = max(1, min(12, os.cpu_count() or 1))
    log(f"batched: CPU oracle, 256 systems on {workers} processes")
    t0 = time.perf_counter()
    with multiprocessing.get_context("fork").Pool(workers) as pool:
        stepsn = sum(pool.map(_det, range(len(systems))))
    dtn = time.perf_counter() - t0
    return dict(value=round(steps1 / dt1, 1), unit="system-steps/s", cores=1, kind="oracle",
                sample=f"systems 0-{sample - 1} of the same batch, 10k steps each, single-threaded, {dt1:.1f} s",
                multi_core=dict(value=round(stepsn / dtn, 1), cores=workers,
                                sample=f"all 256 systems, one per task, {dtn:.1f} s"))


def large_line(cpu=None, tune=True, cache=None):
    import synth
    from paper_1104_1824_amd import snp

    s = synth.config_system(5, 0)
    log("large m=4096 uint16, automatic path, depth 3, cap 4e6")
    w = Walk(s, snp.SNP_PATH_AUTO, 4000000, 3, False, 1 << 22, 12000001, profile=1, tune=tune, cache=cache)
    results, dt = w.timed(3, 1)
    w.close()
    new = results[-1]["n_configs"] - 1
    line = dict(workload=LARGE_WORKLOAD, value=round(3 * new / dt, 1), unit="configs/s",
                ms_per_step=round(dt / 3 * 1e3, 3), levels=results[-1]["level_sizes"].tolist(), dtype="uint16",
                twins=totals(results, "twins"), expanded=totals(results, "expanded"), tuning=w.tuning,
                int8_passes=totals(results, "int8_chunks"), passes=totals(results, "chunks"))
    line.update(hbm_roofline(results, "k_expand_int8", s.m * 2 + ENTRY_BYTES, s.m * 2, workload="large"))
    line["mfma"] = mfma_util(results)
    line["cpu_baseline"] = cpu
    return line


SECONDARY = {"plain_sparse": plain_line, "batched": batched_line, "large": large_line, "delays": delays_line}
CPU_BASELINES = {"dense": cpu_dense, "plain_sparse": cpu_plain, "batched": cpu_batched, "large": cpu_large,
                 "delays": cpu_delays}


def copy_calibration(nbytes=1 << 30, reps=5):
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.add(src, 0, out=dst)  # one elementwise kernel: reads and writes nbytes
    torch.cuda.synchronize()
    log(f"copy calibration: {reps} launches, each reads {nbytes} B and writes {nbytes} B")


def hbm_check(nbytes=2 << 30, reps=10):
    """What plain torch kernels reach on this GPU (context for the rooflines,
    which use the published 8 TB/s): a fill (writes only) and a copy (reads and
    writes), each timed with HIP events on the current stream."""
    import torch

    a = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()

    def timed(fn):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / reps / 1e3

    tf = timed(lambda: a.fill_(3))
    tc = timed(lambda: b.copy_(a))
    print(json.dumps({"hbm_check": {"bytes": nbytes, "fill_ms": round(tf * 1e3, 4),
                                    "fill_write_gbs": round(nbytes / tf / 1e9, 1), "copy_ms": round(tc * 1e3, 4),
                                    "copy_read_write_gbs": round(2 * nbytes / tc / 1e9, 1)}}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the plain-sparse / batched / large lines")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's built-in launch settings (no autotuning before the timed walks)")
    ap.add_argument("--tuning-cache", default=None,
                    help="JSON tuning cache: settings recorded there for a workload are used without tuning, "
                         "new ones are recorded")
    ap.add_argument("--only", choices=sorted(SECONDARY) + ["dense"],
                    help="run only this workload (no CPU baseline) and print its line")
    ap.add_argument("--batch-largest", action="store_true",
                    help="with --only batched: run the workload's largest system alone")
    ap.add_argument("--hbm-check", action="store_true",
                    help="time a 2 GiB fill and copy (what plain kernels reach on this GPU) and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reads 1 GiB, writes 1 GiB) five times, to scale "
                         "FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X, so --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.hbm_check:
        hbm_check()
        return
    # the CPU oracle runs first, before this process touches the GPU (its
    # process pool is forked from here)
    cpus = {}
    if not args.no_cpu_baseline and not args.only:
        for name, fn in CPU_BASELINES.items():
            if name != "dense" and args.no_secondary:
                continue
            log(f"{name}: CPU oracle")
            cpus[name] = fn()
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.only and args.only != "dense":
        kw = dict(largest=args.batch_largest) if args.only == "batched" else dict(tune=not args.no_tune,
                                                                                  cache=args.tuning_cache)
        print(json.dumps({args.only: SECONDARY[args.only](**kw)}), flush=True)
        return
    s, results, dt = run_dense(args.steps, args.warmup, not args.no_tune, args.tuning_cache)
    if args.only == "dense":
        print(json.dumps(dict(ms_per_step=round(dt / args.steps * 1e3, 4),
                              **hbm_roofline(results, "k_expand_int8", s.m * 4 + ENTRY_BYTES, s.m * 4,
                                             workload="dense"))), flush=True)
        return
    new = results[-1]["n_configs"] - 1
    rl = hbm_roofline(results, "k_expand_int8", s.m * 4 + ENTRY_BYTES, s.m * 4, workload="dense")
    sparse = run_dense_sparse(tune=not args.no_tune)
    ms = dt / args.steps * 1e3
    secondary = None
    if not args.no_secondary:
        secondary = {name: fn(cpu=cpus.get(name), **({} if name == "batched" else
                                                      dict(tune=not args.no_tune, cache=args.tuning_cache)))
                     for name, fn in SECONDARY.items()}
    cpu = cpus.get("dense")
    line = {
        "metric": METRIC,
        "value": round(args.steps * new / dt, 1),
        "unit": "configs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {
            "workload": DENSE_WORKLOAD,
            "levels": results[-1]["level_sizes"].tolist(),
            "new_configs_per_step": new,
            "path": "int8 matrix cores (int32 accumulation, int32 rows)",
            "tuning": results[-1].get("tuning"),
            "parallelism": "single GPU",
        },
        "roofline": rl["roofline"],
        "dominant_kernel": rl["dominant_kernel"],
        "mfma": mfma_util(results),
        "vs_plain_sparse": dict(sparse, speedup=round(sparse["ms_per_walk"] / ms, 2)),
        "cpu_baseline": cpu,
        "secondary": secondary,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
