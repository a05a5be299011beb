"""The int8 matrix-core form of C + S.M (reference child + D . M_V on MFMA)
against the oracle, on the same seeded inputs as the sparse form: bit-exact."""
import numpy as np
import pytest

import synth
from paper_1104_1824_amd import snp
from tests.conftest import read_golden
from tests.gpu_helpers import assert_same_bfs, gpu_bfs, note

pytestmark = pytest.mark.gpu

INT8 = snp.SNP_PATH_INT8


def cfg(row):
    return "-".join(str(int(x)) for x in row)


def test_int8_paper_printed_run(gpu, oracle_mod):
    note("int8: paper example")
    ex = synth.paper_example()
    g = gpu_bfs(ex, expand_max_count=9, out_capacity=256, path=INT8)
    assert [cfg(x) for x in g["rows"]] == read_golden("paper_allgenck.txt")
    assert all(st["path_used"] == INT8 for st in g["level_stats"] if st["chunks"])
    assert_same_bfs(g, oracle_mod.bfs(ex, expand_max_count=9))


@pytest.mark.parametrize("seed", range(100))
def test_int8_tiny_plain(gpu, oracle_mod, seed):
    note(f"int8: tiny plain seed {seed}")
    s = synth.config_system(1, seed)
    assert_same_bfs(gpu_bfs(s, max_depth=8, out_capacity=4096, chunk=4096, path=INT8),
                    oracle_mod.bfs(s, max_depth=8))


@pytest.mark.parametrize("seed", range(5))
def test_int8_plain_sparse_full(gpu, oracle_mod, seed):
    note(f"int8: plain sparse seed {seed}, full size")
    s = synth.config_system(2, seed)
    g = gpu_bfs(s, max_depth=1000, frontier_cap=100000, stop_at_cap=True, out_capacity=400000, path=INT8)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=1000, frontier_cap=100000, stop_at_cap=True))


@pytest.mark.parametrize("seed", range(3))
def test_int8_dense_recipe(gpu, oracle_mod, seed):
    note(f"int8: dense recipe m=512 seed {seed}, cap 3000, depth 3")
    s = synth.config_system(3, seed)
    g = gpu_bfs(s, max_depth=3, frontier_cap=3000, out_capacity=10000, path=INT8)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=3, frontier_cap=3000))


def test_int8_large_recipe(gpu, oracle_mod):
    note("int8: large recipe m=4096 u16 seed 0, cap 300, depth 2")
    s = synth.config_system(5, 0)
    g = gpu_bfs(s, max_depth=2, frontier_cap=300, out_capacity=1000, path=INT8)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=2, frontier_cap=300))


def test_int8_hash_collisions_and_chunks(gpu, oracle_mod):
    s = synth.config_system(2, 2)
    want = oracle_mod.bfs(s, max_depth=1000, frontier_cap=20000, stop_at_cap=True)
    for chunk, mask in ((4096, 0), (5000, 0), (0, 0xF00000000000000F)):
        note(f"int8: chunk {chunk} hash mask {mask:#x}")
        g = gpu_bfs(s, max_depth=1000, frontier_cap=20000, stop_at_cap=True, out_capacity=60000, chunk=chunk,
                    hash_mask=mask, path=INT8)
        assert_same_bfs(g, want)


def test_auto_path_matches(gpu, oracle_mod):
    for cid, seed, kw in ((2, 4, dict(max_depth=1000, frontier_cap=5000, stop_at_cap=True)),
                          (3, 1, dict(max_depth=3, frontier_cap=2000))):
        note(f"auto path: recipe {cid} seed {seed}")
        s = synth.config_system(cid, seed)
        assert_same_bfs(gpu_bfs(s, out_capacity=20000, path=snp.SNP_PATH_AUTO, **kw), oracle_mod.bfs(s, **kw))


def test_int8_range_fallback(gpu, oracle_mod):
    """A production of 200 does not fit int8: INT8 falls back to the sparse form."""
    s = synth.config_system(1, 17)
    rules = [(n, i, j, c, 200 if k == 0 else p) for k, (n, i, j, c, p) in enumerate(s.rules())]
    big = synth.make_system(s.m, rules, list(zip(s.syn_src, s.syn_dst)), s.c0)
    note("int8 range fallback")
    g = gpu_bfs(big, max_depth=5, out_capacity=4096, path=INT8)
    assert all(st["int8_fallback"] == 1 and st["path_used"] == snp.SNP_PATH_SPARSE
               for st in g["level_stats"] if st["parents"])
    assert_same_bfs(g, oracle_mod.bfs(big, max_depth=5))


@pytest.mark.parametrize("kmax", [1, 5, 16])
def test_int8_per_child_segments(gpu, oracle_mod, kmax):
    """Segments over int8_max_k rule columns take the per-child sparse form
    inside the int8 kernel (twin skip included); results do not change."""
    from tests.test_gpu_parity import twin_system

    for seed in range(0, 40, 3):
        s = synth.config_system(1, seed)
        note(f"int8 per-child segments kmax {kmax}: tiny seed {seed}")
        assert_same_bfs(gpu_bfs(s, max_depth=8, out_capacity=4096, chunk=4096, path=INT8, int8_max_k=kmax),
                        oracle_mod.bfs(s, max_depth=8))
    tw = twin_system()
    for kw in (dict(), dict(child_budget=3), dict(frontier_cap=2, stop_at_cap=True)):
        note(f"int8 per-child segments kmax {kmax}: twins {kw}")
        assert_same_bfs(gpu_bfs(tw, max_depth=12, out_capacity=4096, path=INT8, int8_max_k=kmax, **kw),
                        oracle_mod.bfs(tw, max_depth=12, **kw))
    s = synth.config_system(3, 2)
    note(f"int8 per-child segments kmax {kmax}: dense recipe seed 2")
    assert_same_bfs(gpu_bfs(s, max_depth=2, frontier_cap=1500, out_capacity=4000, path=INT8, int8_max_k=kmax),
                    oracle_mod.bfs(s, max_depth=2, frontier_cap=1500))


def test_int8_at_the_largest_m(gpu, oracle_mod):
    """m = 4608 (the most neurons a system may have) fits the int8 form's LDS
    with 64-column tiles; m = 4096 takes 128-column tiles."""
    for m in (4608, 4096):
        s = synth.config_system(5, 1, m=m)
        note(f"int8: large recipe m={m} u16 seed 1, cap 200, depth 2")
        g = gpu_bfs(s, max_depth=2, frontier_cap=200, out_capacity=1000, path=INT8)
        assert all(st["path_used"] == INT8 and st["int8_fallback"] == 0 for st in g["level_stats"] if st["chunks"])
        assert_same_bfs(g, oracle_mod.bfs(s, max_depth=2, frontier_cap=200))
