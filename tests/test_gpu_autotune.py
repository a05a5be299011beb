"""The autotuner and its cache: settings picked by timing whole walks never
change results (the walk after tuning, and walks under a sweep of explicit
settings, equal the oracle's), and a second handle of the same workload finds
the settings in the cache."""
import json

import pytest

import synth
from paper_1104_1824_amd import snp
from tests.gpu_helpers import assert_same_bfs, dev_dtype, gpu_bfs, note, to_device_rows
from tests.test_gpu_autopath import ring_choice

pytestmark = pytest.mark.gpu

CASES = {
    # one neuron per lane (m = 64)
    "plain": (lambda: synth.config_system(2, 1), dict(frontier_cap=5000, chunk=1 << 14), 3),
    # int8 matrix cores (m = 512)
    "dense": (lambda: synth.config_system(3, 0), dict(frontier_cap=2000, chunk=1 << 13, path=snp.SNP_PATH_INT8), 3),
    # sparse form (m = 100, out-degree 1)
    "ring": (lambda: ring_choice(), dict(chunk=1 << 13, path=snp.SNP_PATH_SPARSE), 10),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_autotune_then_cache(gpu, oracle_mod, tmp_path, name):
    import torch

    make, opts, depth = CASES[name]
    s = make()
    want = oracle_mod.bfs(s, max_depth=depth, frontier_cap=opts.get("frontier_cap", 0))
    cap = len(want.rows) + 16
    cache = str(tmp_path / "tuning.json")
    note(f"autotune {name}")
    h = snp.snp_load(s, max_rows=cap, **opts)
    try:
        c0 = to_device_rows(s, s.c0)
        out = torch.empty((cap, s.m), dtype=dev_dtype(s), device="cuda")
        best = snp.snp_autotune(h, c0, depth, out, cap, cache)
        assert best["ms"] > 0
        assert snp.snp_get_tuning(h) == {k: best[k] for k in ("chunk", "int8_tiles", "sparse_run")}
    finally:
        h.close()
    entries = json.load(open(cache))["entries"]
    assert len(entries) == 1
    (key, rec), = entries.items()
    assert key.startswith("gfx") and rec["chunk"] == best["chunk"]
    # a new handle of the same workload finds the settings; the walk is unchanged
    note(f"{name}: walk with the cached settings")
    h2 = snp.snp_load(s, max_rows=cap, **opts)
    try:
        assert snp.snp_load_tuning(h2, cache, depth)
        assert snp.snp_get_tuning(h2)["chunk"] == best["chunk"]
        assert not snp.snp_load_tuning(h2, cache, depth + 1)  # another depth: another key
    finally:
        h2.close()
    g = gpu_bfs(s, max_depth=depth, out_capacity=cap, tuning=best, **opts)
    assert_same_bfs(g, want)


@pytest.mark.parametrize("tuning", [dict(chunk=4096, int8_tiles=1), dict(chunk=5000, int8_tiles=16),
                                    dict(chunk=0, int8_tiles=64), dict(chunk=4100, sparse_run=1),
                                    dict(chunk=8192, sparse_run=1024)])
def test_explicit_settings_do_not_change_results(gpu, oracle_mod, tuning):
    for name in sorted(CASES):
        make, opts, depth = CASES[name]
        s = make()
        note(f"settings {tuning} on {name}")
        want = oracle_mod.bfs(s, max_depth=depth, frontier_cap=opts.get("frontier_cap", 0))
        g = gpu_bfs(s, max_depth=depth, out_capacity=len(want.rows) + 16, tuning=tuning, **opts)
        assert_same_bfs(g, want)


def test_tuning_rejects_bad_values_and_foreign_files(gpu, tmp_path):
    s = synth.config_system(1, 3)
    h = snp.snp_load(s, max_rows=64, chunk=8192)
    try:
        for bad in (dict(chunk=8193), dict(int8_tiles=65), dict(sparse_run=-1)):
            with pytest.raises(snp.SnpError) as e:
                snp.snp_set_tuning(h, **bad)
            assert e.value.status == snp.SNP_ERR_INVALID
        other = tmp_path / "other.json"
        other.write_text('{"something": "else"}\n')
        with pytest.raises(snp.SnpError) as e:
            snp.snp_load_tuning(h, str(other), 3)
        assert e.value.status == snp.SNP_ERR_INVALID
        assert other.read_text() == '{"something": "else"}\n'
        assert not snp.snp_load_tuning(h, str(tmp_path / "missing.json"), 3)
    finally:
        h.close()
