"""Keys-first passes of the int8 form: keys, visited set and flags first, then
every row once, each new one straight to its place in the row store, then a
row check of every child taken for a repeat.  The walk must equal the oracle's
and the staged form's (every row staged, the commit copying the new ones)
whether the check passes or a pass is redone.  These walks are small, so
keys-first is forced (stage_rows=-1); by default it runs only where a pass's
rows reach 64 MiB."""
import pytest

import synth
from paper_1104_1824_amd import snp
from tests.gpu_helpers import assert_same_bfs, gpu_bfs, note
from tests.test_gpu_parity import twin_system

pytestmark = pytest.mark.gpu

INT8 = snp.SNP_PATH_INT8


KF = -1  # stage_rows: always keys-first


def redone(g):
    return sum(st["redone"] for st in g["level_stats"])


def same_walk(a, b):
    assert a["level_sizes"].tolist() == b["level_sizes"].tolist()
    assert (a["rows"] == b["rows"]).all()
    assert a["parent"].tolist() == b["parent"].tolist() and a["tindex"].tolist() == b["tindex"].tolist()


@pytest.mark.parametrize("seed", range(3))
def test_dense_recipe_against_staged_and_oracle(gpu, oracle_mod, seed):
    s = synth.config_system(3, seed)
    kw = dict(max_depth=3, frontier_cap=3000)
    note(f"keys-first: dense recipe seed {seed}")
    g = gpu_bfs(s, out_capacity=10000, path=INT8, stage_rows=KF, **kw)
    assert redone(g) == 0
    assert sum(st["keys_first"] for st in g["level_stats"]) == sum(st["chunks"] for st in g["level_stats"])
    assert all(st["path_used"] == INT8 for st in g["level_stats"] if st["chunks"])
    assert_same_bfs(g, oracle_mod.bfs(s, **kw))
    note(f"staged: dense recipe seed {seed}")
    same_walk(g, gpu_bfs(s, out_capacity=10000, path=INT8, stage_rows=1, **kw))


@pytest.mark.parametrize("mask", [0xF00000000000000F, 0xFF000000000000FF, 0x0001000000000FFF])
def test_forced_tag_matches_are_redone(gpu, oracle_mod, mask):
    """With few key bits many keys meet entries of other configurations: the
    row check fails, the pass is redone staged, and the walk is unchanged."""
    s = synth.config_system(2, 2)
    kw = dict(max_depth=1000, frontier_cap=20000, stop_at_cap=True)
    note(f"keys-first: plain sparse seed 2 on int8, hash mask {mask:#x}")
    g = gpu_bfs(s, out_capacity=60000, hash_mask=mask, path=INT8, chunk=4096, stage_rows=KF, **kw)
    assert redone(g) > 0
    assert_same_bfs(g, oracle_mod.bfs(s, **kw))


def test_full_keys_need_no_redo(gpu, oracle_mod):
    s = synth.config_system(2, 2)
    kw = dict(max_depth=1000, frontier_cap=20000, stop_at_cap=True)
    note("keys-first: plain sparse seed 2 on int8, full keys, chunks of 4096")
    g = gpu_bfs(s, out_capacity=60000, path=INT8, chunk=4096, stage_rows=KF, **kw)
    assert redone(g) == 0
    assert_same_bfs(g, oracle_mod.bfs(s, **kw))


@pytest.mark.parametrize("kw", [dict(child_budget=3), dict(frontier_cap=2, stop_at_cap=True), dict(frontier_cap=5),
                                dict(expand_max_count=2)])
def test_twins_caps_and_budgets(gpu, oracle_mod, kw):
    tw = twin_system()
    for mask in (0, 0xF0000000000000F0):
        note(f"keys-first: twins {kw}, mask {mask:#x}")
        g = gpu_bfs(tw, max_depth=12, out_capacity=4096, path=INT8, hash_mask=mask, stage_rows=KF, **kw)
        assert_same_bfs(g, oracle_mod.bfs(tw, max_depth=12, **kw))


@pytest.mark.parametrize("seed", range(0, 60, 4))
def test_tiny_with_masks(gpu, oracle_mod, seed):
    s = synth.config_system(1, seed)
    for mask in (0, 0x3):
        note(f"keys-first: tiny seed {seed}, mask {mask:#x}")
        assert_same_bfs(gpu_bfs(s, max_depth=8, out_capacity=4096, chunk=4096, path=INT8, hash_mask=mask,
                                stage_rows=KF),
                        oracle_mod.bfs(s, max_depth=8))


def test_overflow_in_a_keys_first_pass(gpu, oracle_mod):
    note("keys-first: uint16 overflow on int8")
    s = synth.make_system(2, [(1, 1, 1, 1, 1)], [(1, 0)], [65535, 1], count_type="u16")
    with pytest.raises(snp.SnpError) as e:
        gpu_bfs(s, max_depth=2, out_capacity=16, path=INT8, stage_rows=KF)
    assert e.value.status == snp.SNP_ERR_OVERFLOW
    note("keys-first: int32 at the edge on int8")
    s = synth.make_system(2, [(1, 1, 1, 1, 1)], [(1, 0)], [2**31 - 2, 1])
    assert_same_bfs(gpu_bfs(s, max_depth=3, out_capacity=16, path=INT8, stage_rows=KF),
                    oracle_mod.bfs(s, max_depth=3))


def test_large_recipe_against_staged(gpu, oracle_mod):
    s = synth.config_system(5, 0)
    kw = dict(max_depth=2, frontier_cap=300)
    note("keys-first: large recipe m=4096 u16, cap 300")
    g = gpu_bfs(s, out_capacity=1000, path=INT8, stage_rows=KF, **kw)
    assert_same_bfs(g, oracle_mod.bfs(s, **kw))
    same_walk(g, gpu_bfs(s, out_capacity=1000, path=INT8, stage_rows=1, **kw))


def test_automatic_choice(gpu, oracle_mod):
    """stage_rows 0: a pass takes keys-first where its chunk's rows reach
    64 MiB (the level's 45K-child pass of 2 KiB rows here; passes of 2^14
    children do not), staged below."""
    s = synth.config_system(3, 1)
    kw = dict(max_depth=1, frontier_cap=40000)
    want = oracle_mod.bfs(s, **kw)
    for chunk, keys in ((1 << 16, True), (1 << 14, False)):
        note(f"automatic keys-first: dense recipe seed 1, chunk {chunk}")
        g = gpu_bfs(s, out_capacity=60000, path=INT8, chunk=chunk, **kw)
        assert_same_bfs(g, want)
        kf = sum(st["keys_first"] for st in g["level_stats"])
        assert (kf > 0) == keys, (chunk, kf)
