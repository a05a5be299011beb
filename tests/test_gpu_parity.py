"""Parity of the HIP path (through the C ABI) with the CPU oracle: element by
element on the same seeded inputs; all integer, so bit-exact."""
import numpy as np
import pytest

import oracle
import synth
from paper_1104_1824_amd import snp
from tests.conftest import read_golden
from tests.gpu_helpers import assert_same_bfs, gpu_bfs, note, to_device_rows, from_device_rows, dev_dtype

pytestmark = pytest.mark.gpu

SPARSE = snp.SNP_PATH_SPARSE


def cfg(row):
    return "-".join(str(int(x)) for x in row)


def test_paper_printed_run(gpu, oracle_mod):
    note("paper example, expand_max_count=9")
    ex = synth.paper_example()
    g = gpu_bfs(ex, expand_max_count=9, out_capacity=256)
    assert [cfg(x) for x in g["rows"]] == read_golden("paper_allgenck.txt")
    assert g["stop_reason"] == 0
    assert_same_bfs(g, oracle_mod.bfs(ex, expand_max_count=9))


def test_textbook_reading(gpu, oracle_mod):
    note("paper example, textbook reading")
    ex = synth.paper_example(True)
    assert_same_bfs(gpu_bfs(ex, out_capacity=64), oracle_mod.bfs(ex))


def test_paper_depth_limited(gpu, oracle_mod):
    ex = synth.paper_example()
    for d in (0, 1, 2, 7, 30):
        note(f"paper example depth {d}")
        assert_same_bfs(gpu_bfs(ex, max_depth=d, out_capacity=512), oracle_mod.bfs(ex, max_depth=d))


@pytest.mark.parametrize("seed", range(100))
def test_tiny_plain(gpu, oracle_mod, seed):
    note(f"tiny plain seed {seed}")
    s = synth.config_system(1, seed)
    assert_same_bfs(gpu_bfs(s, max_depth=8, out_capacity=4096, chunk=4096), oracle_mod.bfs(s, max_depth=8))


@pytest.mark.parametrize("seed", range(5))
def test_plain_sparse_small_cap(gpu, oracle_mod, seed):
    note(f"plain sparse seed {seed}, cap 3000")
    s = synth.config_system(2, seed)
    g = gpu_bfs(s, max_depth=1000, frontier_cap=3000, stop_at_cap=True, out_capacity=20000)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=1000, frontier_cap=3000, stop_at_cap=True))


@pytest.mark.parametrize("seed", range(5))
def test_plain_sparse_full(gpu, oracle_mod, seed):
    """The plain-sparse workload at full size: BFS until a level reaches 1e5."""
    note(f"plain sparse seed {seed}, full size")
    s = synth.config_system(2, seed)
    g = gpu_bfs(s, max_depth=1000, frontier_cap=100000, stop_at_cap=True, out_capacity=400000)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=1000, frontier_cap=100000, stop_at_cap=True))


@pytest.mark.parametrize("seed", range(5))
def test_plain_sparse_bench_options(gpu, oracle_mod, seed):
    """The plain-sparse workload with exactly the options the bench times
    (sparse path, chunks of 2^17, expansion timing events on)."""
    note(f"plain sparse seed {seed}, bench options")
    s = synth.config_system(2, seed)
    g = gpu_bfs(s, max_depth=1000, frontier_cap=100000, stop_at_cap=True, out_capacity=200000, max_rows=200000,
                chunk=1 << 17, profile=1)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=1000, frontier_cap=100000, stop_at_cap=True))


def test_auto_path_choice(gpu, oracle_mod):
    """AUTO takes the one-neuron-per-lane sparse form where it applies (m <= 64,
    in-degree <= 16: the tiny and plain-sparse workloads) and the int8 matrix
    cores on the dense workload."""
    for cid, seed, kw, want in ((1, 5, dict(max_depth=8), SPARSE),
                                (2, 0, dict(max_depth=1000, frontier_cap=20000, stop_at_cap=True), SPARSE),
                                (3, 0, dict(max_depth=2, frontier_cap=2000), snp.SNP_PATH_INT8)):
        note(f"auto path choice: recipe {cid} seed {seed}")
        s = synth.config_system(cid, seed)
        g = gpu_bfs(s, out_capacity=50000, path=snp.SNP_PATH_AUTO, **kw)
        assert_same_bfs(g, oracle_mod.bfs(s, **kw))
        assert all(x["path_used"] == want for x in g["level_stats"] if x["chunks"]), cid


@pytest.mark.parametrize("path", [snp.SNP_PATH_SPARSE, snp.SNP_PATH_INT8])
def test_deterministic_walk(gpu, oracle_mod, path):
    """deterministic: one child per configuration (the first spiking vector),
    i.e. the single-branch trajectory up to its first repeat or halting."""
    cases = [(synth.paper_example(), dict(max_depth=40)), (synth.paper_example(True), dict()),
             (synth.paper_example(True), dict(c0=[0, 1, 1]))]
    cases += [(synth.config_system(1, sd), dict(max_depth=60)) for sd in range(0, 40, 3)]
    cases += [(synth.config_system(2, 1), dict(max_depth=200)), (synth.config_system(3, 0), dict(max_depth=30))]
    for s, kw in cases:
        note(f"deterministic walk {s.name} {kw} path {path}")
        g = gpu_bfs(s, out_capacity=512, deterministic=True, path=path, **kw)
        want = oracle_mod.bfs(s, deterministic=True, **kw)
        assert_same_bfs(g, want)
        assert set(g["level_sizes"].tolist()) == {1}


def test_chunk_invariance(gpu, oracle_mod):
    s = synth.config_system(2, 1)
    want = oracle_mod.bfs(s, max_depth=1000, frontier_cap=20000, stop_at_cap=True)
    for chunk in (4096, 5000, 65536, 0):
        note(f"chunk invariance chunk={chunk}")
        g = gpu_bfs(s, max_depth=1000, frontier_cap=20000, stop_at_cap=True, out_capacity=60000, chunk=chunk)
        assert_same_bfs(g, want)


def test_many_scan_tiles(gpu, oracle_mod):
    """Chunks of more than 1024 scan tiles (over 2^20 children) take the
    separate scan of tile counts; smaller ones sum them inside the commit."""
    s = synth.config_system(2, 0)
    want = oracle_mod.bfs(s, max_depth=3, frontier_cap=1200000, stop_at_cap=True)
    assert want.level_sizes.tolist() == [1, 128, 48384, 1200000]
    for chunk in (1 << 21, 0):
        note(f"plain seed 0, cap 1.2e6, depth 3, chunk={chunk}")
        g = gpu_bfs(s, max_depth=3, frontier_cap=1200000, stop_at_cap=True, out_capacity=1300000, chunk=chunk)
        # the last level's first chunk is sized for 1.2e6 new rows: above 2^20
        assert g["level_stats"][2]["expanded"] > (1 << 20)
        assert_same_bfs(g, want)


@pytest.mark.parametrize("seed", [0, 7, 19, 42])
def test_hash_collisions(gpu, oracle_mod, seed):
    """A 4-bit hash makes nearly every probe a tag match: full-row compares
    must keep the result exact."""
    note(f"hash mask 0xF, tiny seed {seed}")
    s = synth.config_system(1, seed)
    g = gpu_bfs(s, max_depth=8, out_capacity=4096, chunk=4096, hash_mask=0xF)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=8))
    note(f"hash mask 0xF00000000000000F, plain seed {seed % 5}")
    s2 = synth.config_system(2, seed % 5)
    g2 = gpu_bfs(s2, max_depth=3, frontier_cap=400, out_capacity=4096, hash_mask=0xF00000000000000F)
    assert_same_bfs(g2, oracle_mod.bfs(s2, max_depth=3, frontier_cap=400))
    # 16 home slots and 16 tags for about a thousand rows: probes meet entries
    # with their tag whose rows differ (a tiny system may have too few rows for
    # that, so the count is checked here)
    assert sum(x["collisions"] for x in g2["level_stats"]) > 0


def test_dense_recipe_small_cap(gpu, oracle_mod):
    note("dense recipe m=512 seed 0, cap 3000, depth 3")
    s = synth.config_system(3, 0)
    g = gpu_bfs(s, max_depth=3, frontier_cap=3000, out_capacity=10000)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=3, frontier_cap=3000))


def test_large_recipe_small_cap(gpu, oracle_mod):
    note("large recipe m=4096 u16 seed 0, cap 300, depth 2")
    s = synth.config_system(5, 0)
    g = gpu_bfs(s, max_depth=2, frontier_cap=300, out_capacity=1000)
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=2, frontier_cap=300))


def test_budget_and_cap(gpu, oracle_mod):
    ex = synth.paper_example()
    note("budget 1")
    assert_same_bfs(gpu_bfs(ex, child_budget=1, out_capacity=16), oracle_mod.bfs(ex, child_budget=1))
    note("cap 1 stop")
    assert_same_bfs(gpu_bfs(ex, frontier_cap=1, stop_at_cap=True, out_capacity=16),
                    oracle_mod.bfs(ex, frontier_cap=1, stop_at_cap=True))
    for seed in (3, 11, 25, 40):
        note(f"cap truncation tiny seed {seed}")
        s = synth.config_system(1, seed)
        assert_same_bfs(gpu_bfs(s, max_depth=5, frontier_cap=2, out_capacity=64, chunk=4096),
                        oracle_mod.bfs(s, max_depth=5, frontier_cap=2))


def test_out_capacity_error(gpu):
    note("out capacity too small")
    ex = synth.paper_example()
    with pytest.raises(snp.SnpError) as e:
        gpu_bfs(ex, expand_max_count=9, out_capacity=10, max_rows=10)
    assert e.value.status == snp.SNP_ERR_CAPACITY


def test_overflow(gpu, oracle_mod):
    note("uint16 overflow")
    s = synth.make_system(2, [(1, 1, 1, 1, 1)], [(1, 0)], [65535, 1], count_type="u16")
    with pytest.raises(snp.SnpError) as e:
        gpu_bfs(s, max_depth=2, out_capacity=16)
    assert e.value.status == snp.SNP_ERR_OVERFLOW
    note("int32 overflow")
    s = synth.make_system(2, [(1, 1, 1, 1, 3)], [(1, 0)], [2**31 - 2, 1])
    with pytest.raises(snp.SnpError) as e:
        gpu_bfs(s, max_depth=2, out_capacity=16)
    assert e.value.status == snp.SNP_ERR_OVERFLOW
    note("int32 at the edge, no overflow")
    s = synth.make_system(2, [(1, 1, 1, 1, 1)], [(1, 0)], [2**31 - 2, 1])
    assert_same_bfs(gpu_bfs(s, max_depth=3, out_capacity=16), oracle_mod.bfs(s, max_depth=3))


def test_bad_c0(gpu, oracle_mod):
    """A C0 count outside the count type's range is an overflow error, whether
    or not a level runs before it is read; the handle stays usable."""
    import torch

    s = synth.config_system(1, 3)
    bad = np.asarray(s.c0, dtype=np.int64).copy()
    bad[s.m // 2] = -1
    h = snp.snp_load(s, path=snp.SNP_PATH_SPARSE, max_rows=1 << 12)
    try:
        out = torch.empty((1 << 12, s.m), dtype=torch.int32, device="cuda")
        for depth in (0, 1, 4, -1):
            note(f"bad C0, max_depth {depth}")
            with pytest.raises(snp.SnpError) as e:
                snp.snp_run(h, to_device_rows(s, bad), depth, out, 1 << 12)
            assert e.value.status == snp.SNP_ERR_OVERFLOW and "C0" in e.value.message
        with pytest.raises(snp.SnpError) as e:
            snp.snp_reset(h, to_device_rows(s, bad))
        assert e.value.status == snp.SNP_ERR_OVERFLOW and "C0" in e.value.message
        note("good C0 on the same handle")
        res = snp.snp_run(h, to_device_rows(s, s.c0), 4, out, 1 << 12)
        want = oracle_mod.bfs(s, max_depth=4)
        assert res["level_sizes"].tolist() == want.level_sizes.tolist()
        assert np.array_equal(from_device_rows(s, out[:res["n_configs"]]), want.rows)
    finally:
        h.close()


def test_all_halting(gpu, oracle_mod):
    note("zero configuration halts")
    ex = synth.paper_example()
    g = gpu_bfs(ex, c0=[0, 0, 0], out_capacity=8)
    o = oracle_mod.bfs(ex, c0=[0, 0, 0])
    assert_same_bfs(g, o)
    assert g["stop_reason"] == 1  # ALL_HALTING


def test_expand_api(gpu, oracle_mod):
    """snp_reset + snp_expand driven level by level equals the oracle's levels."""
    import torch

    for seed in (0, 5, 17, 63):
        note(f"expand api tiny seed {seed}")
        s = synth.config_system(1, seed)
        o = oracle_mod.bfs(s, max_depth=6)
        h = snp.snp_load(s, path=SPARSE, max_rows=4096, chunk=4096)
        try:
            snp.snp_reset(h, to_device_rows(s, s.c0))
            frontier = to_device_rows(s, [s.c0])
            for k in range(1, o.n_levels):
                nxt = torch.empty((256, s.m), dtype=dev_dtype(s), device="cuda")
                par = torch.empty(256, dtype=torch.int64, device="cuda")
                chi = torch.empty(256, dtype=torch.int64, device="cuda")
                n, st = snp.snp_expand(h, frontier, frontier.shape[0], nxt, 256, par, chi)
                assert n == int(o.level_sizes[k])
                assert from_device_rows(s, nxt[:n]).tolist() == o.level(k).tolist()
                off = int(o.level_sizes[:k].sum())
                prev_off = int(o.level_sizes[: k - 1].sum())
                assert (par[:n].cpu().numpy() + prev_off).tolist() == o.parent[off: off + n].tolist()
                assert chi[:n].cpu().numpy().tolist() == o.tindex[off: off + n].tolist()
                frontier = nxt[:n].clone()
        finally:
            h.close()


def test_expand_errors_and_rollback(gpu, oracle_mod):
    import torch

    s = synth.config_system(2, 0)
    h = snp.snp_load(s, path=SPARSE, max_rows=1 << 15)
    try:
        note("expand before reset")
        f = to_device_rows(s, [s.c0])
        nxt = torch.empty((512, s.m), dtype=torch.int32, device="cuda")
        with pytest.raises(snp.SnpError) as e:
            snp.snp_expand(h, f, 1, nxt, 512)
        assert e.value.status == snp.SNP_ERR_INVALID
        snp.snp_reset(h, f[0])
        note("overlapping frontier and next")
        with pytest.raises(snp.SnpError) as e:
            snp.snp_expand(h, nxt[:1], 1, nxt, 512)
        assert e.value.status == snp.SNP_ERR_INVALID
        note("next capacity too small, then retry")
        small = torch.empty((10, s.m), dtype=torch.int32, device="cuda")
        with pytest.raises(snp.SnpError) as e:
            snp.snp_expand(h, f, 1, small, 10)
        assert e.value.status == snp.SNP_ERR_CAPACITY
        n, _ = snp.snp_expand(h, f, 1, nxt, 512)   # the failed call left nothing recorded
        o = oracle_mod.bfs(s, max_depth=1)
        assert n == int(o.level_sizes[1])
        assert from_device_rows(s, nxt[:n]).tolist() == o.level(1).tolist()
        note("empty frontier")
        n, st = snp.snp_expand(h, f, 0, small, 10)
        assert n == 0 and st["parents"] == 0
        note("frontier already visited")
        n, st = snp.snp_expand(h, f, 1, small, 10)
        assert n == 0 and st["enumerated"] == st["children_total"]
    finally:
        h.close()


def test_nondefault_stream(gpu, oracle_mod):
    import torch

    note("handle on a side stream")
    s = synth.config_system(2, 3)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        g = gpu_bfs(s, max_depth=3, frontier_cap=1000, out_capacity=8192, stream=side)
    torch.cuda.synchronize()
    assert_same_bfs(g, oracle_mod.bfs(s, max_depth=3, frontier_cap=1000))


@pytest.mark.parametrize("path", [snp.SNP_PATH_SPARSE, snp.SNP_PATH_INT8])
def test_caps_budgets_many_seeds(gpu, oracle_mod, path):
    """Small caps and budgets cut levels in the middle of a parent's children:
    truncation, enumeration counts, halting counts and stop reasons agree."""
    for seed in range(0, 100, 3):
        s = synth.config_system(1, seed)
        for kw in (dict(frontier_cap=1), dict(frontier_cap=3, stop_at_cap=True), dict(child_budget=2),
                   dict(child_budget=5, frontier_cap=2)):
            note(f"path {path} tiny seed {seed} {kw}")
            assert_same_bfs(gpu_bfs(s, max_depth=6, out_capacity=256, chunk=4096, path=path, **kw),
                            oracle_mod.bfs(s, max_depth=6, **kw))


def test_table_rebuilds(gpu, oracle_mod):
    """Many capped levels leave tombstones (truncated children) until the visited
    set is rebuilt from the row store; results stay exact."""
    s = synth.config_system(2, 0)
    for path in (snp.SNP_PATH_SPARSE, snp.SNP_PATH_INT8):
        note(f"table rebuilds, path {path}")
        g = gpu_bfs(s, max_depth=30, frontier_cap=10, out_capacity=400, max_rows=400, chunk=4096, path=path)
        assert_same_bfs(g, oracle_mod.bfs(s, max_depth=30, frontier_cap=10))


def twin_system():
    """Neurons whose applicable rules share (c, p): children picking a later twin
    repeat an earlier child (identical rows of M_Pi, Definition 2)."""
    rules = [(0, 1, 1, 1, 1), (0, 2, 0, 1, 1), (0, 1, 2, 1, 1), (0, 3, 0, 2, 1),
             (1, 1, 1, 1, 1), (1, 1, 0, 1, 1), (1, 2, 1, 2, 0),
             (2, 1, 1, 1, 2), (2, 1, 1, 1, 2), (3, 1, 1, 1, 1)]
    syn = [(0, 1), (1, 2), (2, 0), (2, 3), (3, 0), (0, 2)]
    return synth.make_system(4, rules, syn, [3, 2, 1, 1], name="twins")


def twin_children(oracle_mod, system, parent):
    """Children of `parent` that fire the later of two applicable rules of one
    neuron with equal (c, p), counted from the oracle's spiking vectors and a
    regex test of applicability (the definition of E = a^i(a^j)*)."""
    import re

    def applies(k, n):
        i, j, c = int(system.rule_i[k]), int(system.rule_j[k]), int(system.rule_c[k])
        return n >= c and re.fullmatch(f"a{{{i}}}(?:a{{{j}}})*", "a" * n) is not None

    _, _, psi = oracle_mod.children(system, parent, max_out=1)
    if psi == 0:
        return 0
    _, S, _ = oracle_mod.children(system, parent, max_out=psi)
    later = np.zeros(len(system.rule_i), dtype=bool)
    for k in range(len(system.rule_i)):
        n = int(system.rule_neuron[k])
        if not applies(k, int(parent[n])):
            continue
        for q in range(k):
            if (int(system.rule_neuron[q]) == n and applies(q, int(parent[n]))
                    and system.rule_c[q] == system.rule_c[k] and system.rule_p[q] == system.rule_p[k]):
                later[k] = True
    return int(np.count_nonzero((S[:, later] != 0).any(axis=1)))


@pytest.mark.parametrize("path", [snp.SNP_PATH_SPARSE, snp.SNP_PATH_INT8])
def test_twin_rules(gpu, oracle_mod, path):
    s = twin_system()
    for kw in (dict(), dict(child_budget=3), dict(child_budget=7, frontier_cap=4), dict(frontier_cap=5),
               dict(frontier_cap=2, stop_at_cap=True)):
        note(f"twin rules, path {path}, {kw}")
        g = gpu_bfs(s, max_depth=12, out_capacity=4096, chunk=4096, path=path, **kw)
        want = oracle_mod.bfs(s, max_depth=12, **kw)
        assert_same_bfs(g, want)
        if not kw:  # no level cut short: every child of every parent is computed
            bounds = np.concatenate([[0], np.cumsum(want.level_sizes)])
            for d, st in enumerate(g["level_stats"][: len(want.level_sizes)]):
                if st["parents"] == 0:
                    continue
                rows = want.rows[bounds[d]: bounds[d + 1]]
                assert st["twins"] == sum(twin_children(oracle_mod, s, r) for r in rows), d


def hub_system(m=24, seed=5):
    """Every neuron feeds neuron 0 (in-degree m - 1 > 16): small m on the
    general expansion kernel rather than the one-neuron-per-lane kernel."""
    base = synth.config_system(1, seed)
    rules = []
    for n in range(m):
        rules.append((n, 1, 1, 1, 1))
        if n % 3 == 0:
            rules.append((n, 2, 1, 2, 1))
        if n % 4 == 1:
            rules.append((n, 1, 0, 1, 0))
    syn = [(n, 0) for n in range(1, m)] + [(0, n) for n in range(1, m, 2)] + [(n, n + 1) for n in range(1, m - 1)]
    c0 = [(3 * n + int(base.c0[n % base.m])) % 4 for n in range(m)]
    return synth.make_system(m, rules, syn, c0, name="hub")


@pytest.mark.parametrize("path", [snp.SNP_PATH_SPARSE, snp.SNP_PATH_INT8])
def test_high_in_degree(gpu, oracle_mod, path):
    s = hub_system()
    for kw in (dict(frontier_cap=3000), dict(frontier_cap=500, stop_at_cap=True), dict(child_budget=777)):
        note(f"hub system (in-degree 23), path {path}, {kw}")
        assert_same_bfs(gpu_bfs(s, max_depth=6, out_capacity=20000, chunk=4096, path=path, **kw),
                        oracle_mod.bfs(s, max_depth=6, **kw))


@pytest.mark.parametrize("path", [snp.SNP_PATH_SPARSE, snp.SNP_PATH_INT8])
def test_uint16_counts_small_m(gpu, oracle_mod, path):
    """uint16 rows on the small-m kernels (plain-sparse recipe re-typed)."""
    for seed in (0, 3):
        s = synth.config_system(2, seed)
        u = synth.make_system(s.m, s.rules(), list(zip(s.syn_src, s.syn_dst)), s.c0, count_type="u16")
        note(f"uint16 plain sparse seed {seed}, path {path}")
        kw = dict(max_depth=1000, frontier_cap=20000, stop_at_cap=True)
        assert_same_bfs(gpu_bfs(u, out_capacity=60000, path=path, **kw), oracle_mod.bfs(u, **kw))


@pytest.mark.parametrize("path", [snp.SNP_PATH_SPARSE, snp.SNP_PATH_INT8])
def test_halting_counts_after_cut(gpu, oracle_mod, path):
    """Levels cut by the cap with halting parents past the cut: the halting
    statistic counts parents up to the last enumerated child's parent."""
    for seed in (49, 93, 97):
        s = synth.config_system(1, seed)
        note(f"halting after cut: tiny seed {seed}, path {path}")
        assert_same_bfs(gpu_bfs(s, max_depth=8, out_capacity=256, chunk=4096, path=path, frontier_cap=3),
                        oracle_mod.bfs(s, max_depth=8, frontier_cap=3))


def wide_psi_system(m):
    """Every neuron holds 2 applicable rules (c = 1 and c = 2, p = 1) and 2
    in-synapses, so Psi(C0) = 2^m, far beyond 2^32, and child t has a closed
    form: neuron j fires its second rule iff bit m-1-j of t is set (Algorithm 2
    II-3, neuron 1 most significant), giving C0[n] + 2 - 1 - bit_n(t)."""
    rules = []
    for n in range(m):
        rules += [(n, 1, 1, 1, 1), (n, 2, 1, 2, 1)]
    syn = [(n, (n + 1) % m) for n in range(m)] + [(n, (n + 7) % m) for n in range(m)]
    c0 = [5 + (n % 3) for n in range(m)]
    return synth.make_system(m, rules, syn, c0, name=f"wide_psi_m{m}")


@pytest.mark.parametrize("m,path", [(40, snp.SNP_PATH_SPARSE), (80, snp.SNP_PATH_SPARSE), (40, snp.SNP_PATH_INT8)])
def test_psi_beyond_32_bits(gpu, m, path):
    """Parents with Psi > 2^32 (64-bit digit decomposition).  The oracle
    enumerates every child to count Psi, so at 2^m children these runs are
    checked against the closed form instead: level 1 is children 0 .. cap-1
    of C0 (all distinct), level 2 the same children of level 1's first row."""
    s = wide_psi_system(m)
    cap = 3000
    note(f"Psi = 2^{m}, path {path}")
    g = gpu_bfs(s, max_depth=2, frontier_cap=cap, stop_at_cap=False, out_capacity=1 + 2 * cap, path=path)
    assert g["level_sizes"].tolist() == [1, cap, cap]
    st = g["level_stats"]
    # children counts saturate at 2^62
    assert st[0]["children_total"] == min(2 ** m, 2 ** 62)
    assert st[0]["enumerated"] == cap and st[0]["halting_parents"] == 0
    assert st[1]["enumerated"] == cap
    c0 = np.asarray(s.c0, dtype=np.int64)
    t = np.arange(cap, dtype=np.int64)
    bits = (t[:, None] >> (m - 1 - np.arange(m))[None, :]) & 1
    lvl1 = c0[None, :] + 1 - bits
    lvl2 = lvl1[0][None, :] + 1 - bits
    assert np.array_equal(g["rows"][1:1 + cap], lvl1)
    assert np.array_equal(g["rows"][1 + cap:], lvl2)
    assert g["parent"].tolist() == [-1] + [0] * cap + [1] * cap
    assert g["tindex"].tolist() == [-1] + list(range(cap)) * 2
