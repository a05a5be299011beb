"""Helpers of the GPU tests: run the HIP library through its C ABI on torch
buffers and compare with the oracle on the same seeded inputs."""
import sys
import time

import numpy as np

import oracle
from paper_1104_1824_amd import snp


def note(msg):
    """Name the case on stdout before each GPU step (a fault then names it)."""
    print(f"[gpu] {time.strftime('%H:%M:%S')} {msg}", flush=True)
    sys.stdout.flush()


def dev_dtype(system):
    import torch

    # uint16 counts travel as int16 bit patterns; the library reads the bytes
    return torch.int16 if system.count_type == "u16" else torch.int32


def to_device_rows(system, rows):
    import torch

    a = np.asarray(rows, dtype=np.int64)
    if system.count_type == "u16":
        a = a.astype(np.uint16).view(np.int16)
    else:
        a = a.astype(np.int32)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def from_device_rows(system, t):
    a = t.cpu().numpy()
    if system.count_type == "u16":
        a = a.view(np.uint16)
    return a.astype(np.int64)


def gpu_bfs(system, max_depth=-1, out_capacity=1 << 16, c0=None, with_prov=True, tuning=None, **opts):
    import torch

    opts.setdefault("path", snp.SNP_PATH_SPARSE)
    opts.setdefault("max_rows", out_capacity)
    h = snp.snp_load(system, **opts)
    try:
        if tuning:
            snp.snp_set_tuning(h, **{k: v for k, v in tuning.items() if k != "ms"})
        c0 = np.asarray(system.c0 if c0 is None else c0, dtype=np.int64)
        if c0.shape[0] < h.m:  # extra row entries (output spike train, delay states) start at 0
            c0 = np.concatenate([c0, np.zeros(h.m - c0.shape[0], dtype=np.int64)])
        c0t = to_device_rows(system, c0)
        out = torch.empty((out_capacity, h.m), dtype=dev_dtype(system), device="cuda")
        par = torch.empty(out_capacity, dtype=torch.int64, device="cuda") if with_prov else None
        chi = torch.empty(out_capacity, dtype=torch.int64, device="cuda") if with_prov else None
        res = snp.snp_run(h, c0t, max_depth, out, out_capacity, parent_of=par, child_of=chi)
        n = res["n_configs"]
        res["rows"] = from_device_rows(system, out[:n])
        if with_prov:
            res["parent"] = par[:n].cpu().numpy()
            res["tindex"] = chi[:n].cpu().numpy()
        return res
    finally:
        h.close()


def assert_same_bfs(gres, ores, check_stats=True):
    """Bit-exact comparison of a GPU run with the oracle's run."""
    assert gres["level_sizes"].tolist() == ores.level_sizes.tolist()
    assert gres["stop_reason"] == ores.stop_reason, (gres["stop_reason"], ores.stop_reason)
    assert gres["rows"].shape == ores.rows.shape
    bad = np.nonzero((gres["rows"] != ores.rows).any(axis=1))[0]
    assert bad.size == 0, f"{bad.size} rows differ, first at {bad[:5].tolist()}"
    if "parent" in gres:
        assert gres["parent"].tolist() == ores.parent.tolist()
        assert gres["tindex"].tolist() == ores.tindex.tolist()
    if check_stats:
        st = gres["level_stats"]
        L = len(ores.level_sizes)
        assert [s["enumerated"] for s in st[:L]] == ores.enumerated.tolist()
        assert [s["halting_parents"] for s in st[:L]] == ores.halting.tolist()
        # children that repeat an earlier configuration: enumerated minus new
        new = [int(ores.level_sizes[k + 1]) if k + 1 < L else 0 for k in range(L)]
        dup = [int(e) - n if int(e) else 0 for e, n in zip(ores.enumerated.tolist(), new)]
        assert [s["duplicates"] for s in st[:L]] == dup
