"""Deterministic batched mode (one launch for many systems) against the oracle:
final configuration, halting step, first repeat, steps computed and the
trajectory checksum, all bit-exact."""
import numpy as np
import pytest

import synth
from paper_1104_1824_amd import snp
from tests.gpu_helpers import from_device_rows, note

pytestmark = pytest.mark.gpu


def ring(m, c0_pos=0):
    """One spike travelling round a ring: C_k = e_{k mod m}, first repeat at step m."""
    rules = [(n, 1, 1, 1, 1) for n in range(m)]
    syn = [(n, (n + 1) % m) for n in range(m)]
    c0 = [0] * m
    c0[c0_pos] = 1
    return synth.make_system(m, rules, syn, c0, name=f"ring{m}")


def path(m):
    """One spike along a path that leaves at its end: C_m = 0, which halts."""
    rules = [(n, 1, 1, 1, 1) for n in range(m)]
    syn = [(n, n + 1) for n in range(m - 1)]
    c0 = [0] * m
    c0[0] = 1
    return synth.make_system(m, rules, syn, c0, name=f"path{m}")


def run_batch(systems, steps, detect=True, threads=0):
    import torch

    b = snp.snp_batch_load(systems, threads=threads)
    try:
        off = snp.snp_batch_offsets(b)
        dt = torch.int16 if systems[0].count_type == "u16" else torch.int32
        c0 = np.concatenate([np.asarray(s.c0, dtype=np.int64) for s in systems])
        if systems[0].count_type == "u16":
            c0 = c0.astype(np.uint16).view(np.int16)
        c0_t = torch.from_numpy(c0.astype(np.int16 if systems[0].count_type == "u16" else np.int32)).cuda()
        final = torch.empty(int(off[-1]), dtype=dt, device="cuda")
        res = snp.snp_batch_run(b, c0_t, steps, final, detect)
        fin = from_device_rows(systems[0], final)
        res["final"] = [fin[off[k]: off[k + 1]] for k in range(len(systems))]
        return res
    finally:
        b.close()


def check_against_oracle(oracle_mod, systems, steps, res, detect=True):
    for k, s in enumerate(systems):
        d = oracle_mod.deterministic(s, steps)
        assert res["final"][k].tolist() == d.final.tolist(), (k, s.name)
        assert int(res["halt_step"][k]) == d.halt_step, (k, s.name)
        assert int(res["steps_done"][k]) == d.steps_done, (k, s.name)
        assert int(res["digest"][k]) == d.digest, (k, s.name)
        if detect:
            assert int(res["first_repeat"][k]) == d.first_repeat, (k, s.name)


def test_batch_constructed_repeats_and_halts(gpu, oracle_mod):
    ex, tb = synth.paper_example(), synth.paper_example(True)
    tb_halt = synth.make_system(tb.m, tb.rules(), list(zip(tb.syn_src, tb.syn_dst)), [0, 1, 1])
    systems = [ex, tb, tb_halt, ring(5), ring(64), ring(100), ring(128), ring(200, 7), path(150), path(64)]
    for steps in (0, 1, 63, 64, 65, 300):
        note(f"batch constructed systems, steps {steps}")
        res = run_batch(systems, steps)
        check_against_oracle(oracle_mod, systems, steps, res)
    res = run_batch(systems, 300)
    assert res["first_repeat"].tolist()[3:8] == [5, 64, 100, 128, 200]
    assert res["halt_step"].tolist()[8:] == [150, 64]


def test_batch_tiny_seeds(gpu, oracle_mod):
    systems = [synth.config_system(1, s) for s in range(64)]
    note("batch of 64 tiny systems, 500 steps")
    check_against_oracle(oracle_mod, systems, 500, run_batch(systems, 500))


def test_batch_uneven_recipe_sample(gpu, oracle_mod):
    """Systems of the batched recipe (m in [16, 1024]) for 1500 steps."""
    systems = synth.batched_systems(0, 24)
    note("batch of 24 uneven systems, 1500 steps")
    check_against_oracle(oracle_mod, systems, 1500, run_batch(systems, 1500))


def golden_batch():
    from tests.golden import make_golden

    head, data = make_golden.read_table(make_golden.BATCH_FILE)
    assert int(head["steps"]) == 10000 and len(data) == 256
    return make_golden, data


def test_batch_full_recipe_golden(gpu):
    """The full batched workload (256 systems, 10k steps) in one launch, as the
    bench runs it; every system against the oracle-written golden lines."""
    make_golden, data = golden_batch()
    systems = synth.batched_systems(0, 256)
    note("batch of 256 uneven systems, 10000 steps")
    res = run_batch(systems, 10000)
    for k, line in enumerate(data):
        seed, m, fin, halt, rep, done, dig = line
        assert int(seed) == k and int(m) == systems[k].m
        got = make_golden.sha(np.ascontiguousarray(res["final"][k].astype("<i4")).tobytes())
        assert got == fin, k
        assert int(res["halt_step"][k]) == int(halt), k
        assert int(res["first_repeat"][k]) == int(rep), k
        assert int(res["steps_done"][k]) == int(done), k
        assert int(res["digest"][k]) == int(dig), k


def test_run_batch_entry_point(gpu, oracle_mod):
    """snp_run_batch over handles from snp_load (one row buffer per system)
    equals the oracle, on a first list, a second call with the same list (the
    kept batch), and a different list."""
    import torch

    from tests.gpu_helpers import to_device_rows

    def go(systems, steps):
        hs = [snp.snp_load(s, max_rows=16) for s in systems]
        try:
            c0 = [to_device_rows(s, s.c0) for s in systems]
            fin = [torch.full((s.m,), -1, dtype=torch.int32, device="cuda") for s in systems]
            for rep in range(2):
                note(f"snp_run_batch, {len(systems)} systems, {steps} steps, call {rep}")
                res = snp.snp_run_batch(hs, c0, steps, fin)
                for k, s in enumerate(systems):
                    d = oracle_mod.deterministic(s, steps)
                    assert fin[k].cpu().numpy().tolist() == d.final.tolist(), (rep, k)
                    assert int(res["halt_step"][k]) == d.halt_step
                    assert int(res["first_repeat"][k]) == d.first_repeat
                    assert int(res["digest"][k]) == d.digest
                for f in fin:
                    f.fill_(-1)
        finally:
            for h in hs:
                h.close()

    go(synth.batched_systems(7, 6) + [ring(64), path(30), synth.paper_example()], 500)
    go([synth.config_system(1, sd) for sd in range(12)], 300)


def test_batch_uint16_and_overflow(gpu, oracle_mod):
    systems = [synth.config_system(1, s) for s in range(8)]
    u16 = [synth.make_system(s.m, s.rules(), list(zip(s.syn_src, s.syn_dst)), s.c0, count_type="u16")
           for s in systems]
    note("uint16 batch")
    check_against_oracle(oracle_mod, u16, 200, run_batch(u16, 200))
    note("uint16 overflow")
    # two neurons feeding each other: each consumes 1 and receives 2 per step
    grow = synth.make_system(2, [(0, 1, 1, 1, 2), (1, 1, 1, 1, 2)], [(0, 1), (1, 0)], [65530, 65530],
                             count_type="u16")
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.deterministic(grow, 50)
    with pytest.raises(snp.SnpError) as e:
        run_batch([grow] + u16, 50)
    assert e.value.status == snp.SNP_ERR_OVERFLOW


def test_batch_without_repeat_detection(gpu, oracle_mod):
    systems = [ring(100), synth.paper_example(True), path(70)]
    note("repeat detection off")
    res = run_batch(systems, 250, detect=False)
    check_against_oracle(oracle_mod, systems, 250, res, detect=False)
    assert res["first_repeat"].tolist() == [-1, -1, -1]


@pytest.mark.parametrize("threads", [256, 512, 1024])
def test_batch_every_launch_shape(gpu, oracle_mod, threads):
    """Each fixed launch shape (threads per system; up to 4 neurons per thread)
    gives the oracle's results; the autotuned shape is one of them."""
    systems = synth.batched_systems(3, 12) + [ring(100), path(70), synth.paper_example()]
    systems = [s for s in systems if s.m <= 4 * threads]
    note(f"batch shape {threads} threads, {len(systems)} systems, 700 steps")
    check_against_oracle(oracle_mod, systems, 700, run_batch(systems, 700, threads=threads))


def test_batch_graph_replays(gpu, oracle_mod):
    """The recorded launch is replayed on later calls (with other GPU work in
    between); every replay matches the first, eager-built result and the oracle."""
    import torch

    systems = synth.batched_systems(5, 10) + [ring(64), path(40)]
    b = snp.snp_batch_load(systems)
    try:
        off = snp.snp_batch_offsets(b)
        c0 = torch.from_numpy(np.concatenate([s.c0 for s in systems]).astype(np.int32)).cuda()
        fin = torch.empty(int(off[-1]), dtype=torch.int32, device="cuda")
        results = []
        for rep, steps in enumerate((300, 300, 300, 130, 300)):
            note(f"graph replay {rep}, steps {steps}")
            junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated work between replays
            torch.cuda.synchronize()
            fin.fill_(-1)
            res = snp.snp_batch_run(b, c0, steps, fin)
            res["final"] = fin.cpu().numpy().copy()
            results.append((steps, res))
            assert float(junk) == float(junk)
        th, npt = snp.snp_batch_shape(b)
        assert th in (256, 512, 1024) and npt in (1, 2, 4)
    finally:
        b.close()
    base = results[0][1]
    for steps, res in results:
        if steps == 300:
            for k in ("halt_step", "first_repeat", "steps_done", "digest", "final"):
                assert np.array_equal(res[k], base[k]), k
    for steps in (300, 130):
        res = [r for s_, r in results if s_ == steps][0]
        fin_rows = [res["final"][off[k]: off[k + 1]] for k in range(len(systems))]
        for k, s in enumerate(systems):
            d = oracle_mod.deterministic(s, steps)
            assert fin_rows[k].tolist() == d.final.tolist()
            assert int(res["digest"][k]) == d.digest and int(res["first_repeat"][k]) == d.first_repeat


def periodic_rules_system(seed, m=96):
    """Rules with the periods the kernel's residue table takes (j dividing 24)
    and some it does not (5, 7, 9), thresholds i and c up to 40, productions up
    to 3: counts pass the thresholds at different steps, some neurons never use
    the table."""
    rng = synth.SplitMix64((7 << 32) | seed)
    js = (0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 24)
    rules = []
    for n in range(m):
        for _ in range(rng.uniform(1, 4)):
            i = rng.uniform(1, 40)
            rules.append((n, i, rng.choice(js), rng.uniform(1, i), rng.uniform(0, 3)))
    syn = []
    for n in range(m):
        seen = set()
        while len(seen) < rng.uniform(1, 6):
            d = rng.below(m)
            if d != n:
                seen.add(d)
        syn.extend((n, d) for d in sorted(seen))
    c0 = [rng.uniform(0, 60) for _ in range(m)]
    return synth.make_system(m, rules, syn, c0, name=f"periodic_s{seed}")


@pytest.mark.parametrize("threads", [256, 1024])
def test_batch_residue_table_periods(gpu, oracle_mod, threads):
    systems = [periodic_rules_system(s) for s in range(12)]
    for steps in (1, 40, 700):
        note(f"batch residue-table periods, {threads} threads, steps {steps}")
        res = run_batch(systems, steps, threads=threads)
        check_against_oracle(oracle_mod, systems, steps, res)


def many_rules_system(seed, m=70):
    """Neurons with 5 to 16 rules whose first ones need large counts (so the
    fired rule is often past the fourth, and a 16-rule neuron has no table for
    small counts), plus a hub neuron with 60 in-synapses (past the 32 sources a
    lane holds in registers); m = 70 leaves slots past m in the last wave."""
    rng = synth.SplitMix64((11 << 32) | seed)
    rules = []
    for n in range(m):
        k = 16 if n % 7 == 0 else rng.uniform(5, 12)
        for q in range(k):
            if q < k - 3:  # thresholds that the counts reach only now and then
                i = rng.uniform(8, 40)
                rules.append((n, i, rng.choice((0, 1, 2, 3, 5)), rng.uniform(1, i), rng.uniform(0, 3)))
            else:  # late rules that apply to small counts
                i = rng.uniform(1, 3)
                rules.append((n, i, rng.choice((0, 1, 2)), rng.uniform(1, i), rng.uniform(0, 2)))
    syn = set()
    hub = m - 1
    for n in range(m):
        for _ in range(rng.uniform(1, 4)):
            d = rng.below(m)
            if d != n:
                syn.add((n, d))
    for n in range(60):
        if n != hub:
            syn.add((n, hub))
    c0 = [rng.uniform(0, 30) for _ in range(m)]
    return synth.make_system(m, rules, sorted(syn), c0, name=f"many_rules_s{seed}")


@pytest.mark.parametrize("threads", [256, 512, 1024])
def test_batch_many_rules_and_a_hub(gpu, oracle_mod, threads):
    systems = [many_rules_system(s) for s in range(6)]
    assert max(np.bincount(s.syn_dst).max() for s in systems) > 32
    for steps in (1, 37, 500):
        note(f"batch many rules and a hub, {threads} threads, steps {steps}")
        check_against_oracle(oracle_mod, systems, steps, run_batch(systems, steps, threads=threads))


@pytest.mark.parametrize("seed", [300, 307, 314])
def test_batch_random_sweep(gpu, oracle_mod, seed):
    """Systems of the batched recipe from other seeds, every launch shape that
    fits, step counts that end inside a 4-step group and inside a 64-step batch
    (odd counts leave the odd production buffer last)."""
    systems = synth.batched_systems(seed, 4)
    rng = synth.SplitMix64((13 << 32) | seed)
    for threads in (256, 512, 1024):
        fit = [s for s in systems if s.m <= 4 * threads]
        for steps in (rng.uniform(1, 7), rng.uniform(65, 130), rng.uniform(200, 600)):
            note(f"batch random sweep seed {seed}, {threads} threads, {len(fit)} systems, steps {steps}")
            check_against_oracle(oracle_mod, fit, steps, run_batch(fit, steps, threads=threads))
