"""SN P systems with delays on the GPU (the variant the paper leaves to the work
it cites, Section 2.1): walks through the C ABI equal the oracle's row for row,
with the delay states (wait, pend) after the counts; bit-exact."""
import numpy as np
import pytest

import synth
from paper_1104_1824_amd import snp
from synth.systems import make_system, with_delays
from tests.gpu_helpers import assert_same_bfs, gpu_bfs, note

pytestmark = pytest.mark.gpu

HAND = {
    "chain": make_system(3, [(0, 1, 0, 1, 1, 2), (1, 1, 0, 1, 1, 0)], [(0, 1), (1, 2)], [1, 0, 0]),
    "lost_spike": make_system(3, [(0, 1, 0, 1, 1, 0), (1, 1, 0, 1, 1, 1)], [(0, 1), (1, 2)], [1, 1, 0]),
    "receive_at_send": make_system(3, [(0, 1, 1, 1, 1, 0), (1, 1, 0, 1, 1, 1)], [(0, 1), (1, 2)], [2, 1, 0]),
    "no_fire_at_send": make_system(2, [(0, 1, 1, 1, 1, 1)], [(0, 1)], [2, 0]),
    "delay_choice": make_system(2, [(0, 1, 0, 1, 1, 0), (0, 1, 0, 1, 1, 1)], [(0, 1)], [1, 0]),
}


@pytest.mark.parametrize("name", sorted(HAND))
def test_hand_worked_runs(gpu, oracle_mod, name):
    s = HAND[name]
    note(f"delays, hand-worked run {name}")
    assert_same_bfs(gpu_bfs(s, out_capacity=64), oracle_mod.bfs(s))


@pytest.mark.parametrize("delays", [(2,), (2, 4), (1, 3, 5)])
def test_output_neuron_generates_the_delays(gpu, oracle_mod, delays):
    rules = [(0, 1, 0, 1, 1, 0)] + [(0, 1, 0, 1, 1, d) for d in delays]
    rules += [(1, 1, 0, 1, 1, 0), (2, 1, 0, 1, 1, 0), (2, 2, 0, 2, 1, 0)]
    s = make_system(3, rules, [(0, 2), (1, 2)], [1, 1, 0])
    depth = 2 * max(delays) + 6
    note(f"delays, output neuron, delays {delays}")
    g = gpu_bfs(s, max_depth=depth, out_neuron=3, out_capacity=256)
    want = oracle_mod.bfs(s, max_depth=depth, out_neuron=3)
    assert_same_bfs(g, want)
    assert oracle_mod.generated_numbers(want, 3) == sorted(delays)


@pytest.mark.parametrize("seed", range(40))
def test_tiny_delayed(gpu, oracle_mod, seed):
    s = with_delays(synth.config_system(1, seed), seed, d_max=1 + seed % 4)
    note(f"delays, tiny seed {seed}")
    assert_same_bfs(gpu_bfs(s, max_depth=10, out_capacity=4096, chunk=4096), oracle_mod.bfs(s, max_depth=10))


@pytest.mark.parametrize("seed", range(0, 24, 3))
def test_tiny_delayed_output_neuron(gpu, oracle_mod, seed):
    s = with_delays(synth.config_system(1, seed), seed, d_max=3)
    for out in (1, 2, 3):
        note(f"delays, tiny seed {seed}, output neuron {out}")
        assert_same_bfs(gpu_bfs(s, max_depth=10, out_neuron=out, out_capacity=4096),
                        oracle_mod.bfs(s, max_depth=10, out_neuron=out))


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("count_type", ["i32", "u16"])
def test_plain_sparse_delayed(gpu, oracle_mod, seed, count_type):
    """m = 64, out-degree 4, delays up to 3 on half the rules: BFS until a level
    reaches 20000, in several passes per level (chunks of 4096 children)."""
    s = with_delays(synth.config_system(2, seed), seed, d_max=3)
    s.count_type = count_type
    note(f"delays, plain sparse seed {seed} {count_type}")
    g = gpu_bfs(s, max_depth=1000, frontier_cap=20000, stop_at_cap=True, out_capacity=1 << 17, chunk=4096)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=1000, frontier_cap=20000, stop_at_cap=True, rows_cap=1 << 17))


@pytest.mark.parametrize("seed", range(3))
def test_dense_delayed_budget(gpu, oracle_mod, seed):
    """m = 512, out-degree 64 (rows of about 1400 entries with the delay
    states): the first level under a child budget; the int8 form is asked for
    and falls back to the sparse form."""
    s = with_delays(synth.config_system(3, seed), seed, d_max=3)
    note(f"delays, dense seed {seed}, budget 3000, INT8 requested")
    g = gpu_bfs(s, max_depth=2, child_budget=3000, out_capacity=1 << 14, path=snp.SNP_PATH_INT8)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=2, child_budget=3000, rows_cap=1 << 14))
    assert all(st["int8_fallback"] == 1 for st in g["level_stats"][:1])
    assert all(st["int8_chunks"] == 0 for st in g["level_stats"])


@pytest.mark.parametrize("seed", range(6))
def test_caps_budgets_and_collisions(gpu, oracle_mod, seed):
    s = with_delays(synth.config_system(2, seed, m=12), seed, d_max=2)
    kw = [dict(frontier_cap=50), dict(frontier_cap=40, stop_at_cap=True), dict(child_budget=77),
          dict(expand_max_count=3)]
    for k in kw:
        note(f"delays, m=12 seed {seed}, {k}")
        assert_same_bfs(gpu_bfs(s, max_depth=6, out_capacity=1 << 14, chunk=4096, **k),
                        oracle_mod.bfs(s, max_depth=6, rows_cap=1 << 14, **k))
    note(f"delays, m=12 seed {seed}, hash mask 0xF")
    assert_same_bfs(gpu_bfs(s, max_depth=5, out_capacity=1 << 14, hash_mask=0xF),
                    oracle_mod.bfs(s, max_depth=5, rows_cap=1 << 14))


@pytest.mark.parametrize("seed", range(8))
def test_deterministic_branch(gpu, oracle_mod, seed):
    s = with_delays(synth.config_system(2, seed, m=16), seed, d_max=3)
    note(f"delays, deterministic, m=16 seed {seed}")
    assert_same_bfs(gpu_bfs(s, max_depth=200, deterministic=True, out_capacity=1024),
                    oracle_mod.bfs(s, max_depth=200, deterministic=True))


def test_zero_delays_are_the_plain_system(gpu, oracle_mod):
    """rule_d all 0: no state entries, and the one-neuron-per-lane form runs."""
    s = synth.config_system(2, 1)
    z = with_delays(s, 1, num=0)
    h = snp.snp_load(z, max_rows=1 << 10)
    try:
        assert h.m == s.m
    finally:
        h.close()
    note("zero delays, plain sparse seed 1")
    g = gpu_bfs(z, max_depth=1000, frontier_cap=3000, stop_at_cap=True, out_capacity=20000)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=1000, frontier_cap=3000, stop_at_cap=True))


def test_batched_mode_refuses_delays(gpu):
    s = with_delays(synth.config_system(1, 2), 2, d_max=2)
    assert s.rule_d.any()
    with pytest.raises(snp.SnpError):
        snp.snp_batch_load([s])
    h = snp.snp_load(s, max_rows=64)
    try:
        import torch

        c0 = torch.zeros((h.m,), dtype=torch.int32, device="cuda")
        fin = torch.zeros((h.m,), dtype=torch.int32, device="cuda")
        with pytest.raises(snp.SnpError):
            snp.snp_run_batch([h], [c0], 3, [fin])
    finally:
        h.close()


@pytest.mark.parametrize("tuning", [None, dict(chunk=1 << 15, int8_tiles=0, sparse_run=64),
                                    dict(chunk=1 << 17, int8_tiles=0, sparse_run=4)])
def test_bench_delay_workload(gpu, oracle_mod, tuning):
    """The delays workload exactly as the benchmark times it (sparse path,
    chunks of 2^17 children, expansion timing on, 400000 rows), with the
    built-in launch settings and with settings the tuner can pick."""
    import bench

    s = bench.delay_system()
    note(f"delays bench workload, tuning {tuning}")
    g = gpu_bfs(s, max_depth=1000, frontier_cap=100000, stop_at_cap=True, out_capacity=400000, max_rows=400000,
                chunk=1 << 17, profile=1, tuning=tuning)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=1000, frontier_cap=100000, stop_at_cap=True, rows_cap=1 << 19))
