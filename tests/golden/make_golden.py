"""Write the oracle-computed golden digests of the full-size workloads.

Calls only the CPU oracle (``oracle/``) and the seeded generator (``synth/``);
nothing here touches the GPU library.  Two files are written next to this
script:

* ``dense_m512_s0_walk.txt`` and ``dense_m512_s1_walk.txt`` -- the
  breadth-first walk of the dense workload (m = 512, 3 rules per neuron, p in
  [0, 4], out-degree 64, C0 in [0, 4], int32 counts; seeds 0 and 1), depth 3,
  frontier cap 1e6 per level (Algorithm 1 with
  the children of every configuration in Algorithm 2 order, Equation
  next-config).  The walk's rows are cut into blocks of 1024 consecutive rows
  (global row index, C0 is row 0); every block gets two digests: SHA-256 of the
  rows as little-endian int32, and SHA-256 of the (parent, child index) pairs
  as little-endian int64, interleaved per row.  Each digest is cut to its first
  24 hex digits.
* ``batched_256x10k.txt`` -- the deterministic single-branch run (every neuron
  fires its first applicable rule; Section 2.1 global clock) of the 256
  systems of the batched workload (seeds 0-255), 10,000 steps each: per
  system, SHA-256 (24 hex digits) of the final configuration as little-endian
  int32, the halting step, the first repeat, the steps computed and the
  trajectory checksum.

Usage: ``python tests/golden/make_golden.py [dense|dense1|batched|all]`` (each
dense walk takes a few minutes of one CPU core and about 13 GB of memory).
"""
import hashlib
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

BLOCK = 1024
HEX = 24
DENSE_SEEDS = (0, 1)


def dense_file(seed: int = 0) -> str:
    return os.path.join(HERE, f"dense_m512_s{seed}_walk.txt")


DENSE_FILE = dense_file(0)
BATCH_FILE = os.path.join(HERE, "batched_256x10k.txt")
DENSE_RUN = dict(max_depth=3, frontier_cap=1000000)
BATCH_STEPS = 10000
BATCH_SEEDS = 256


def sha(b: bytes) -> str:
    return hashlib.sha256(b).hexdigest()[:HEX]


def block_digests(rows: np.ndarray, parent: np.ndarray, tindex: np.ndarray, first_block: int = 0,
                  last_block: int = None):
    """(rows digest, provenance digest) of blocks first_block .. last_block - 1."""
    n = rows.shape[0]
    nb = (n + BLOCK - 1) // BLOCK
    last_block = nb if last_block is None else min(last_block, nb)
    out = []
    for k in range(first_block, last_block):
        a, b = k * BLOCK, min(n, (k + 1) * BLOCK)
        r = np.ascontiguousarray(rows[a:b].astype("<i4"))
        prov = np.empty((b - a, 2), dtype="<i8")
        prov[:, 0] = parent[a:b]
        prov[:, 1] = tindex[a:b]
        out.append((sha(r.tobytes()), sha(prov.tobytes())))
    return out


def read_table(path):
    """(header fields, data lines) of a golden file."""
    head, data = {}, []
    with open(path) as f:
        for ln in f:
            ln = ln.rstrip("\n")
            if ln.startswith("#"):
                if ":" in ln and ln.startswith("# @"):
                    k, v = ln[3:].split(":", 1)
                    head[k.strip()] = v.strip()
                continue
            if ln.strip():
                data.append(ln.split())
    return head, data


def write_dense(seed=0):
    s = synth.config_system(3, seed)
    t0 = time.time()
    res = oracle.bfs(s, rows_cap=3000001, **DENSE_RUN)
    dt = time.time() - t0
    digs = block_digests(res.rows, res.parent, res.tindex)
    with open(dense_file(seed), "w") as f:
        f.write("# Breadth-first walk of the dense workload, computed by the CPU oracle\n")
        f.write("# (written by tests/golden/make_golden.py, which calls only oracle/ and synth/).\n")
        f.write("# System: m=512, 3 rules per neuron, E = a^i (a^j)* with i in [1,4], j in [0,3], c in [1,i],\n")
        f.write(f"# p in [0,4], out-degree 64, C0 in [0,4], int32 counts; seed {seed} of the dense recipe.\n")
        f.write("# Walk: Algorithm 1 (one global visited set, first occurrence kept) with the children of a\n")
        f.write("# configuration in Algorithm 2 step II-3 order, C' = C + S.M (Equation next-config);\n")
        f.write("# depth 3, every level truncated to its first 1e6 new configurations.\n")
        f.write(f"# @levels: {' '.join(str(int(x)) for x in res.level_sizes)}\n")
        f.write(f"# @stop_reason: {res.stop_reason}\n")
        f.write(f"# @enumerated: {' '.join(str(int(x)) for x in res.enumerated)}\n")
        f.write(f"# @halting: {' '.join(str(int(x)) for x in res.halting)}\n")
        f.write(f"# @block_rows: {BLOCK}\n")
        f.write(f"# Each line: block k (rows [{BLOCK}k, {BLOCK}k + {BLOCK}) of the walk, C0 = row 0), SHA-256 of the\n")
        f.write(f"# rows as little-endian int32, SHA-256 of the (parent row, child index) pairs as little-endian\n")
        f.write(f"# int64 (C0: -1, -1), each cut to its first {HEX} hex digits.\n")
        for k, (a, b) in enumerate(digs):
            f.write(f"{k} {a} {b}\n")
    print(f"dense walk, seed {seed}: {res.n_levels} levels {res.level_sizes.tolist()}, {len(digs)} blocks, oracle {dt:.1f} s")


def batch_line(seed):
    s = synth.batched_systems(seed, 1)[0]
    d = oracle.deterministic(s, BATCH_STEPS)
    fin = sha(np.ascontiguousarray(d.final.astype("<i4")).tobytes())
    return f"{seed} {s.m} {fin} {d.halt_step} {d.first_repeat} {d.steps_done} {d.digest}"


def write_batched(workers=8):
    oracle.build(force=False)
    t0 = time.time()
    with Pool(workers) as pool:
        lines = pool.map(batch_line, range(BATCH_SEEDS))
    dt = time.time() - t0
    with open(BATCH_FILE, "w") as f:
        f.write("# Deterministic single-branch runs of the batched workload, computed by the CPU oracle\n")
        f.write("# (written by tests/golden/make_golden.py, which calls only oracle/ and synth/).\n")
        f.write("# Systems: seeds 0-255 of the batched recipe (m in [16,1024], 1-3 rules and out-degree 2-32 per\n")
        f.write("# neuron, int32 counts).  Every neuron fires its first applicable rule at every step (Section 2.1,\n")
        f.write(f"# one rule per neuron on a global clock), C' = C + S.M, for {BATCH_STEPS} steps or until halting.\n")
        f.write(f"# @steps: {BATCH_STEPS}\n")
        f.write("# Each line: seed, m, SHA-256 of the final configuration as little-endian int32 (first 24 hex\n")
        f.write("# digits), halting step, first repeat, steps computed, trajectory checksum (unsigned 64-bit).\n")
        for ln in lines:
            f.write(ln + "\n")
    print(f"batched: {BATCH_SEEDS} systems in {dt:.1f} s ({workers} processes)")


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    oracle.build(force=False)
    if what in ("batched", "all"):
        write_batched()
    if what in ("dense", "all"):
        write_dense(0)
    if what in ("dense1", "all"):
        write_dense(1)
