"""Benchmark: new configurations per second of the breadth-first expansion.

One step is one complete breadth-first walk of the plain-sparse workload
(seeded synthetic system, m = 64 neurons, 2 rules per neuron, out-degree 4,
C0 uniform in [0, 4], int32 counts) from C0 until a level reaches 100,000
configurations: every level runs applicability + Psi, the prefix sum, the
expansion C' = C + S.M, the visited-set insert and the ordered commit, all on
the GPU through the C ABI.  The value is new (deduplicated) configurations
per second over the timed steps; inputs are resident in HBM before timing.

The JSON line also carries the roofline of the dominant kernel (device time
from HIP events recorded by the library on its stream just before and after
each of its launches inside the timed region) and the CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "new configurations/sec (deduped) per BFS step; int8-MFMA/batched vs plain sparse"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
# bytes per child of the one-neuron-per-lane expansion besides its row: key 8,
# parent 4, child index 8, probe slot 4, visited-set entry 8
LANE_CHILD_EXTRA = 32
TWIN_CHILD_BYTES = 12  # a twin child: parent 4 and child index 8 only


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def plain_sparse_workload(seed=0):
    import synth

    return synth.config_system(2, seed), dict(frontier_cap=100000, stop_at_cap=True, max_depth=1000)


def run_gpu(system, run_opts, steps, warmup):
    import torch

    from paper_1104_1824_amd import snp

    cap = 200000
    h = snp.snp_load(system, path=snp.SNP_PATH_SPARSE, frontier_cap=run_opts["frontier_cap"],
                     stop_at_cap=run_opts["stop_at_cap"], max_rows=cap, chunk=1 << 17, profile=1)
    c0 = torch.tensor(system.c0, dtype=torch.int32, device="cuda")
    out = torch.empty((cap, system.m), dtype=torch.int32, device="cuda")
    res = None
    for _ in range(warmup):
        res = snp.snp_run(h, c0, run_opts["max_depth"], out, cap)
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for _ in range(steps):
        results.append(snp.snp_run(h, c0, run_opts["max_depth"], out, cap))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h.close()
    return results, t1 - t0, res


def walk_timing(system, path, cap, depth, stop, chunk, out_cap, reps):
    """Mean time of `reps` complete walks on one path (after one untimed walk)."""
    import numpy as np
    import torch

    from paper_1104_1824_amd import snp

    h = snp.snp_load(system, path=path, frontier_cap=cap, stop_at_cap=stop, max_rows=out_cap, chunk=chunk,
                     profile=2)
    u16 = system.count_type == "u16"
    c0 = np.asarray(system.c0, dtype=np.int64)
    c0 = torch.from_numpy(c0.astype(np.uint16).view(np.int16) if u16 else c0.astype(np.int32)).cuda()
    out = torch.empty((out_cap, system.m), dtype=torch.int16 if u16 else torch.int32, device="cuda")
    snp.snp_run(h, c0, depth, out, out_cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        r = snp.snp_run(h, c0, depth, out, out_cap)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    h.close()
    st = r["level_stats"]
    ns = sum(s_["ns_expand"] for s_ in st)
    expanded = sum(s_["expanded"] for s_ in st)
    twins = sum(s_["twins"] for s_ in st)
    rb = system.m * (2 if u16 else 4)
    # a child writes its row, key, parent and index; a twin child only its
    # parent and index
    moved = (expanded - twins) * (rb + 20) + twins * TWIN_CHILD_BYTES
    return dict(ms_per_walk=round(dt * 1e3, 3), new_configs=int(r["n_configs"] - 1),
                configs_per_s=round((r["n_configs"] - 1) / dt, 1), levels=r["level_sizes"].tolist(),
                expand_us=round(ns / 1e3, 1), expand_gbs=round(moved / max(ns, 1), 1), twins=int(twins),
                stage_us={k: round(sum(s_["ns_" + k] for s_ in st) / 1e3, 1)
                          for k in ("psi", "expand", "insert", "flags", "commit")})


def extra_plain_int8():
    """The plain-sparse workload on the int8 matrix-core form."""
    import synth
    from paper_1104_1824_amd import snp

    log("plain sparse workload, int8 path")
    return walk_timing(synth.config_system(2, 0), snp.SNP_PATH_INT8, 100000, 1000, True, 1 << 17, 200000, 10)


def extra_dense():
    """Dense m=512 workload: the int8 matrix-core form next to the sparse form."""
    import synth
    from paper_1104_1824_amd import snp

    s3 = synth.config_system(3, 0)
    dense = {}
    for name, path, reps in (("int8", snp.SNP_PATH_INT8, 3), ("sparse", snp.SNP_PATH_SPARSE, 1)):
        log(f"dense m=512 workload, {name} path")
        dense[name] = walk_timing(s3, path, 1000000, 3, False, 1 << 20, 3100000, reps)
    dense["speedup_int8_over_sparse"] = round(dense["sparse"]["ms_per_walk"] / dense["int8"]["ms_per_walk"], 2)
    dense["workload"] = ("dense_int8: m=512, 3 rules/neuron (r=1536), p in [0,4] (M entries in [-4,4]), "
                         "out-degree 64, C0 in [0,4], int32; BFS depth 3, frontier_cap 1e6 per level (seed 0)")
    return dense


def extra_large():
    """Large exploration: m=4096, uint16, depth 3, cap 4e6 per level, automatic path."""
    import synth
    from paper_1104_1824_amd import snp

    log("large m=4096 uint16 workload, automatic path, depth 3, cap 4e6")
    # chunks of 2^22 children (34 GB of staged rows): few passes over the long runs of twins
    r = walk_timing(synth.config_system(5, 0), snp.SNP_PATH_AUTO, 4000000, 3, False, 1 << 22, 12000001, 1)
    r["workload"] = ("large: m=4096, 4 rules/neuron (r=16384), out-degree 16, C0 in [0,8], uint16; BFS depth 3, "
                     "frontier_cap 4e6 per level (seed 0)")
    return r


def extra_batched():
    """The batched deterministic launch (256 systems x 10k steps)."""
    import numpy as np
    import torch

    import synth
    from paper_1104_1824_amd import snp

    log("batched deterministic launch, 256 systems x 10k steps")
    systems = synth.batched_systems(0, 256)
    b = snp.snp_batch_load(systems)
    off = snp.snp_batch_offsets(b)
    c0 = torch.from_numpy(np.concatenate([x.c0 for x in systems]).astype(np.int32)).cuda()
    fin = torch.empty(int(off[-1]), dtype=torch.int32, device="cuda")
    snp.snp_batch_run(b, c0, 10000, fin)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        snp.snp_batch_run(b, c0, 10000, fin)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    shape = snp.snp_batch_shape(b)
    b.close()
    return dict(
        workload="batched_uneven: 256 systems, m in [16,1024], 1-3 rules and out-degree 2-32 per neuron, "
                 "10k deterministic steps each, one launch (seeds 0-255)",
        ms_per_launch=round(dt * 1e3, 3), system_steps=256 * 10000,
        system_steps_per_s=round(256 * 10000 / dt, 1),
        threads_per_system=shape[0], neurons_per_thread=shape[1])


EXTRAS = {"plain_sparse_int8_path": extra_plain_int8, "dense_int8": extra_dense, "large": extra_large,
          "batched": extra_batched}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_expand_lane_plain_sparse_m64_traffic.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1104_1824_amd", "csrc", "snp_kernels.hip")


def measured_traffic():
    """HBM bytes per launch of the expansion kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter runs (scaled by the copy calibration), or
    None when the kernel source changed since they were taken."""
    import hashlib

    if not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    for ln in open(TRAFFIC_FILE):
        if ":" in ln and ln.strip().startswith("- `"):
            k, v = ln.strip()[3:].split("`:", 1)
            fields[k.strip()] = v.strip().strip("`")
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if fields.get("kernel_source_sha256") != sha:
        return None
    return int(fields["traffic_bytes_per_launch"])


def roofline(system, results):
    """Roofline of the expansion kernel: its algorithmic bytes over its device
    time.  Algorithmic bytes per launch = children computed x (row bytes written
    + 20 B of per-child key, parent index and child index + 12 B of its
    visited-set probe: the slot index and the entry it writes); parent rows,
    read once per segment of children, and the entry read by the probe's
    compare-and-swap are not counted."""
    rb = system.m * 4
    ns = 0
    launches = 0
    children = 0
    twins = 0
    for r in results:
        for st in r["level_stats"]:
            ns += st["ns_expand"]
            launches += st["chunks"]
            children += st["expanded"]
            twins += st["twins"]
    steps = len(results)
    bytes_expand = (children - twins) * (rb + LANE_CHILD_EXTRA) + twins * TWIN_CHILD_BYTES
    achieved = bytes_expand / max(1, ns)  # bytes per ns = GB/s
    return dict(
        kernel="k_expand_lane",
        bound="hbm",
        achieved=round(achieved, 2),
        peak=HBM_PEAK_GBS,
        unit="GB/s",
        frac=round(achieved / HBM_PEAK_GBS, 4),
        traffic=measured_traffic(),
        bytes_per_launch=round(bytes_expand / max(1, launches)),
        avg_launch_us=round(ns / max(1, launches) / 1e3, 3),
        launches_per_step=launches // max(1, steps),
        expand_us_per_step=round(ns / 1e3 / max(1, steps), 2),
    )


def cpu_baseline(system, run_opts, budget_s=12.0):
    import oracle

    oracle.build(force=False)
    n_new = 0
    runs = 0
    t0 = time.perf_counter()
    while True:
        res = oracle.bfs(system, max_depth=run_opts["max_depth"], frontier_cap=run_opts["frontier_cap"],
                         stop_at_cap=run_opts["stop_at_cap"], rows_cap=1 << 18)
        n_new += int(res.level_sizes[1:].sum())
        runs += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=round(n_new / dt, 1), unit="configs/s", cores=1, kind="oracle",
                sample=f"{runs} complete BFS walks of the same workload (plain sparse seed 0), "
                       f"single-threaded C oracle, {dt:.1f} s")


def copy_calibration(nbytes=1 << 30, reps=5):
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.add(src, 0, out=dst)  # one elementwise kernel: reads and writes nbytes
    torch.cuda.synchronize()
    log(f"copy calibration: {reps} launches, each reads {nbytes} B and writes {nbytes} B")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the int8 / dense / batched side measurements")
    ap.add_argument("--only", choices=sorted(EXTRAS), help="run only this side measurement and print it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reads 1 GiB, writes 1 GiB) five times, to scale "
                         "FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.only:
        print(json.dumps({args.only: EXTRAS[args.only]()}), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library runs on a single MI355X, so --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    system, run_opts = plain_sparse_workload(0)
    log(f"plain sparse seed 0: m={system.m} r={system.r} syn={system.n_syn}; warmup {args.warmup}, steps {args.steps}")
    results, dt, _ = run_gpu(system, run_opts, args.steps, args.warmup)
    new_per_step = results[-1]["n_configs"] - 1
    sizes = results[-1]["level_sizes"].tolist()
    assert all(r["n_configs"] - 1 == new_per_step for r in results)
    value = args.steps * new_per_step / dt
    log(f"levels {sizes}, {new_per_step} new configurations per step, {dt / args.steps * 1e3:.3f} ms/step")
    rl = roofline(system, results)
    log(f"expansion kernel {rl['expand_us_per_step']} us per step")
    extras = None
    if not args.no_extras:
        extras = {name: fn() for name, fn in EXTRAS.items()}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on the same workload")
        cpu = cpu_baseline(system, run_opts)
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "configs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": "plain_sparse: seeded SN P system m=64, 2 rules/neuron (r=128), E=a^i(a^j)* "
                        "i in [1,4] j in [0,3], out-degree 4, C0 in [0,4], int32; BFS until a level "
                        "reaches 1e5 configurations (seed 0)",
            "levels": sizes,
            "new_configs_per_step": new_per_step,
            "path": "sparse",
            "parallelism": "single GPU",
        },
        "roofline": {k: rl[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "dominant_kernel": {k: rl[k] for k in ("kernel", "bytes_per_launch", "avg_launch_us", "launches_per_step",
                                                "expand_us_per_step")},
        "cpu_baseline": cpu,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
