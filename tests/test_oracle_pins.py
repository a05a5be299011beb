"""Pins of the CPU oracle to facts the paper and the mathematics fix.

None of these tests runs the GPU path.  Each pin is chosen so that a plausible
mistake in the oracle (wrong applicability, dropped term of Definition 2, wrong
significance order of the enumeration, a missing dedup, wrong truncation) fails
at least one of them.
"""
import ast
import itertools
import re

import numpy as np
import pytest

import synth
from oracle import alg2
from tests.conftest import read_golden

EX = synth.paper_example()          # exponent k read as "at least k spikes" (E = a^k a*)
EX_TB = synth.paper_example(True)   # exponent k read as exactly a^k (rule form b-3)


def cfg(row):
    return "-".join(str(int(x)) for x in row)


def golden_trace():
    out = {}
    for ln in read_golden("paper_trace.txt"):
        key, val = ln.split(":", 1)
        out[key.strip()] = val.strip()
    return out


# --------------------------------------------------------------------------
# The generator's random source: SplitMix64 (Steele, Lea, Flood 2014).
# --------------------------------------------------------------------------
def test_splitmix64_published_outputs():
    r = synth.SplitMix64(0)
    assert [r.next_u64() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_digest_mixer_is_splitmix64_finaliser(oracle_mod):
    # SplitMix64 output i (seed 0) is the finaliser applied to (i + 1) * gamma
    gamma = 0x9E3779B97F4A7C15
    assert [oracle_mod.mix64((i + 1) * gamma) for i in range(3)] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


# --------------------------------------------------------------------------
# Definition 2 against the matrix printed for the example (Section 2.2) and its
# row-major input file (Section 3.1).
# --------------------------------------------------------------------------
def test_paper_matrix(oracle_mod):
    lines = read_golden("paper_matrix.txt")
    printed = np.array([[int(x) for x in ln.split()] for ln in lines if not ln.startswith("row-major")])
    row_major = [int(x) for x in lines[-1].split(":", 1)[1].split()]
    M = oracle_mod.matrix_dense(EX)
    assert M.tolist() == printed.tolist()
    assert M.reshape(-1).tolist() == row_major
    # the textbook reading changes E only, not M
    assert oracle_mod.matrix_dense(EX_TB).tolist() == printed.tolist()


def test_rule_file_encodes_exponents():
    # rule file "2 2 $ 1 $ 1 2" (Section 4) -> r = [[2, 2], [1], [1, 2]]
    tr = golden_trace()
    groups = [[int(x) for x in part.split()] for part in tr["rules"].split("$")]
    assert groups == ast.literal_eval(tr["r"])
    exps = [[int(EX.rule_i[k]) for k in range(EX.r) if EX.rule_neuron[k] == n] for n in range(EX.m)]
    assert exps == groups


# --------------------------------------------------------------------------
# Applicability against Python's regular-expression engine (an independent
# implementation of L(E)), for E = a^i (a^j)* and the n >= c condition.
# --------------------------------------------------------------------------
def test_applicability_matches_regex(oracle_mod):
    for i in range(1, 7):
        for j in range(0, 6):
            pat = re.compile(f"a{{{i}}}" if j == 0 else f"a{{{i}}}(?:a{{{j}}})*")
            for n in range(0, 30):
                in_lang = pat.fullmatch("a" * n) is not None
                for c in (1, i, i + 1):
                    assert oracle_mod.applicable(n, i, j, c) == (in_lang and n >= c), (n, i, j, c)


# --------------------------------------------------------------------------
# Algorithm 2 on the worked example: intermediates printed in Section 4.2.
# --------------------------------------------------------------------------
def _applies_at_least(n, k):
    return n >= k


def test_alg2_intermediates_at_c0():
    tr = golden_trace()
    r = ast.literal_eval(tr["r"])
    tmp = alg2.step_ii1([2, 1, 1], r, _applies_at_least)
    assert tmp == ast.literal_eval(tr["tmp"])
    assert alg2.psi(tmp) == int(tr["psi"])
    tmp2 = alg2.step_ii2(tmp)
    assert tmp2 == ast.literal_eval(tr["tmp2"])
    assert alg2.step_ii3(tmp2) == ast.literal_eval(tr["tmp3"])


def test_c_oracle_children_at_c0_follow_tmp3(oracle_mod):
    tr = golden_trace()
    rows, S, psi = oracle_mod.children(EX, [2, 1, 1])
    assert psi == int(tr["psi"])
    assert ["".join(str(int(b)) for b in s) for s in S] == ast.literal_eval(tr["tmp3"])
    assert [cfg(x) for x in rows] == ast.literal_eval(tr["after_211"])[1:]


# --------------------------------------------------------------------------
# The printed run (Section 5): all 48 configurations of allGenCk, in order,
# the snapshots printed along the way, and the stop reason.  The run records
# but does not expand configurations holding a two-digit count (reading of the
# printed list: 2-1-10 and 1-1-10 appear, 2-1-11 does not).
# --------------------------------------------------------------------------
def test_paper_printed_run(oracle_mod):
    want = read_golden("paper_allgenck.txt")
    res = oracle_mod.bfs(EX, expand_max_count=9)
    got = [cfg(x) for x in res.rows]
    assert got == want
    assert res.stop_reason == oracle_mod.STOP_EMPTY_FRONTIER
    assert res.level_sizes.tolist() == [1, 2, 4, 6, 6, 6, 5, 5, 5, 5, 2, 1]
    tr = golden_trace()
    for key in ("after_211", "after_212", "after_112"):
        snap = ast.literal_eval(tr[key])
        assert got[: len(snap)] == snap
    # the deepest configuration the run expanded is 1-0-9 (the last one listed)
    assert got[-1] == "1-0-9"


def test_paper_closed_form(oracle_mod):
    """Closed form of the reachable set under "expand only if every count <= N".

    By hand from Definition 2 (reading: rule exponent k means at least k spikes):
    (2,1,k) -> (2,1,k+1), (2,1,k), (1,1,k+1), (1,1,k) [last two need k >= 2 for r5];
    (1,1,k) -> (2,0,k), (2,0,k-1); (2,0,k) -> (1,1,k), (1,1,k-1), (0,1,k), (0,1,k-1);
    (0,1,k) -> (1,0,k), (1,0,k-1); (1,0,k) -> (1,0,k-1), (1,0,k-2); (1,0,0) halts.
    Hence {2-1-k, 1-1-k : 1<=k<=N+1} U {2-0-k, 0-1-k : 1<=k<=N} U {1-0-k : 0<=k<=N},
    5N + 3 configurations (48 for N = 9, the printed run).
    """
    for N in (2, 3, 5, 9, 14):
        res = oracle_mod.bfs(EX, expand_max_count=N)
        got = {cfg(x) for x in res.rows}
        want = set()
        for k in range(1, N + 2):
            want |= {f"2-1-{k}", f"1-1-{k}"}
        for k in range(1, N + 1):
            want |= {f"2-0-{k}", f"0-1-{k}"}
        for k in range(0, N + 1):
            want.add(f"1-0-{k}")
        assert got == want and len(res.rows) == 5 * N + 3


def test_textbook_reading(oracle_mod):
    """Rule form b-3 (E = a^k exactly), worked by hand: 211 -> {212, 112};
    212 -> {212, 112} (seen); 112 -> {201}; 201 -> {111, 011}; 111 -> {201};
    011 -> {101}; 101 -> {100}; 100 has no applicable rule."""
    res = oracle_mod.bfs(EX_TB)
    levels = [[cfg(x).replace("-", "") for x in res.level(k)] for k in range(res.n_levels)]
    assert levels == [["211"], ["212", "112"], ["201"], ["111", "011"], ["101"], ["100"]]
    assert res.stop_reason == oracle_mod.STOP_ALL_HALTING


# --------------------------------------------------------------------------
# Brute force on tiny random systems: every 0/1 vector over the r rules in
# descending binary order (rule 1 = most significant bit), kept when valid
# (one applicable rule per neuron that has one, none elsewhere; applicability
# by regex), child = C + S M with dense integer arithmetic.
# --------------------------------------------------------------------------
def _brute_children(sys, M, C):
    rules = sys.rules()
    app = []
    for (n, i, j, c, p) in rules:
        pat = f"a{{{i}}}" if j == 0 else f"a{{{i}}}(?:a{{{j}}})*"
        app.append(re.fullmatch(pat, "a" * int(C[n])) is not None and C[n] >= c)
    out_rows, out_S = [], []
    r = len(rules)
    for v in range((1 << r) - 1, -1, -1):
        S = [(v >> (r - 1 - k)) & 1 for k in range(r)]
        ok = True
        for n in range(sys.m):
            ks = [k for k in range(r) if rules[k][0] == n]
            fired = [k for k in ks if S[k]]
            if any(not app[k] for k in fired):
                ok = False
                break
            if len(fired) != (1 if any(app[k] for k in ks) else 0):
                ok = False
                break
        if ok:
            out_S.append(S)
            out_rows.append(np.asarray(C, dtype=np.int64) + np.asarray(S, dtype=np.int64) @ M)
    if not any(app):
        return [], []  # halting: no child
    return out_rows, out_S


@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_enumeration(oracle_mod, seed):
    rng = synth.SplitMix64(1000 + seed)
    m = rng.uniform(2, 4)
    counts = [rng.uniform(1, 3) for _ in range(m)]
    while sum(counts) > 10:
        counts[rng.below(m)] = 1
    sys = synth.random_system(rng, m, counts, (1, 3), (0, 1, 2), (0, 1, 2), (1, m - 1), (0, 5))
    M = oracle_mod.matrix_dense(sys)
    seen = 0
    for trial in range(6):
        C = [rng.uniform(0, 6) for _ in range(m)]
        want_rows, want_S = _brute_children(sys, M, C)
        rows, S, psi = oracle_mod.children(sys, C)
        assert psi == len(want_rows)
        assert [list(map(int, x)) for x in rows] == [list(map(int, x)) for x in want_rows]
        assert S.tolist() == want_S
        # the string form of Algorithm 2 lists the same vectors in the same order
        per = [[(int(sys.rule_i[k]), int(sys.rule_j[k]), int(sys.rule_c[k])) for k in range(sys.r)
                if sys.rule_neuron[k] == n] for n in range(m)]
        strings = alg2.spiking_vectors(
            C, per, lambda x, rule: oracle_mod.applicable(x, rule[0], rule[1], rule[2]))
        if psi:
            assert strings == ["".join(str(b) for b in s) for s in want_S]
        seen += psi
    assert seen > 0


# --------------------------------------------------------------------------
# Invariants of a BFS (spike conservation per fired rule, provenance, levels
# pairwise disjoint, first-occurrence order) on tiny-plain systems.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(0, 100, 9))
def test_bfs_invariants(oracle_mod, seed):
    sys = synth.config_system(1, seed)
    res = oracle_mod.bfs(sys, max_depth=8)
    rows = res.rows
    assert len({tuple(x) for x in rows.tolist()}) == len(rows)
    assert (rows >= 0).all()
    outdeg = np.bincount(sys.syn_src, minlength=sys.m)
    for q in range(1, len(rows)):
        par, t = int(res.parent[q]), int(res.tindex[q])
        assert par < q
        crow, S, _ = oracle_mod.children(sys, rows[par], max_out=t + 1)
        assert crow[t].tolist() == rows[q].tolist()
        fired = np.nonzero(S[t])[0]
        delta = sum(-int(sys.rule_c[k]) + int(sys.rule_p[k]) * int(outdeg[sys.rule_neuron[k]]) for k in fired)
        assert int(rows[q].sum() - rows[par].sum()) == delta
    # first-occurrence order: (parent, t) increases along each level
    off = 0
    for k in range(res.n_levels):
        n = int(res.level_sizes[k])
        keys = list(zip(res.parent[off: off + n].tolist(), res.tindex[off: off + n].tolist()))
        assert keys == sorted(keys)
        off += n


# --------------------------------------------------------------------------
# Truncation and budget follow their definitions: a capped level is the first
# `cap` configurations of the uncapped level list that were never recorded,
# in enumeration order.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed,cap", [(3, 2), (11, 3), (25, 1), (40, 4)])
def test_cap_truncation_definition(oracle_mod, seed, cap):
    sys = synth.config_system(1, seed)
    res = oracle_mod.bfs(sys, max_depth=5, frontier_cap=cap)
    recorded = {tuple(res.rows[0].tolist())}
    frontier = [res.rows[0]]
    for k in range(1, res.n_levels):
        want = []
        for par in frontier:
            rows, _, _ = oracle_mod.children(sys, par)
            for x in rows.tolist():
                if tuple(x) not in recorded and x not in want:
                    want.append(x)
        want = want[:cap]
        assert res.level(k).tolist() == want
        recorded |= {tuple(x) for x in want}
        frontier = list(res.level(k))


def _halting_by_regex(sys, C):
    """No rule applies anywhere (applicability by Python's regex engine)."""
    for k in range(sys.r):
        i, j, c = int(sys.rule_i[k]), int(sys.rule_j[k]), int(sys.rule_c[k])
        pat = f"a{{{i}}}" if j == 0 else f"a{{{i}}}(?:a{{{j}}})*"
        n = int(C[int(sys.rule_neuron[k])])
        if n >= c and re.fullmatch(pat, "a" * n):
            return False
    return True


# seeds 49, 93 and 97 with cap 3 have halting parents after a level's cut,
# where "up to the last enumerated child's parent" differs from "all parents"
@pytest.mark.parametrize("seed,kw", [(3, dict(frontier_cap=2)), (8, dict(frontier_cap=3)), (19, dict(child_budget=4)),
                                     (27, dict(child_budget=3, frontier_cap=2)), (33, dict()), (54, dict(frontier_cap=1)),
                                     (49, dict(frontier_cap=3)), (93, dict(frontier_cap=3)), (97, dict(frontier_cap=3))])
def test_level_statistics_definition(oracle_mod, seed, kw):
    """Per expanded level: `enumerated` counts children in canonical order up to
    where the level stopped (the cap-filling child, the budget, or all), and
    `halting` counts parents without an applicable rule up to the parent of the
    last child enumerated (every parent when the level ran to its end)."""
    sys = synth.config_system(1, seed)
    res = oracle_mod.bfs(sys, max_depth=8, **kw)
    cap, budget = kw.get("frontier_cap", 0), kw.get("child_budget", 0)
    recorded = {tuple(res.rows[0].tolist())}
    for k in range(res.n_levels):
        if res.enumerated[k] == 0 and res.halting[k] == 0:
            continue
        frontier = res.level(k)
        enumerated, new, last_par, cut = 0, [], -1, False
        for q, par in enumerate(frontier):
            rows, _, _ = oracle_mod.children(sys, par)
            for x in rows.tolist():
                if budget and enumerated == budget:
                    cut = True
                    break
                enumerated += 1
                last_par = q
                if tuple(x) not in recorded and x not in new:
                    new.append(x)
                    if cap and len(new) == cap:
                        cut = True
                        break
            if cut:
                break
        p_end = last_par + 1 if cut else len(frontier)
        halting = sum(_halting_by_regex(sys, frontier[q]) for q in range(p_end))
        assert int(res.enumerated[k]) == enumerated, (k, enumerated)
        assert int(res.halting[k]) == halting, (k, halting)
        recorded |= {tuple(x) for x in new}


def test_budget_stops_level(oracle_mod):
    res = oracle_mod.bfs(EX, child_budget=1)
    assert [cfg(x) for x in res.rows] == ["2-1-1", "2-1-2"]
    assert res.stop_reason == oracle_mod.STOP_BUDGET
    assert res.enumerated.tolist() == [1, 0]


def test_stop_at_cap(oracle_mod):
    res = oracle_mod.bfs(EX, frontier_cap=1, stop_at_cap=True)
    assert [cfg(x) for x in res.rows] == ["2-1-1", "2-1-2"]
    assert res.stop_reason == oracle_mod.STOP_CAP


def test_overflow_reported(oracle_mod):
    sys = synth.make_system(2, [(1, 1, 1, 1, 1)], [(1, 0)], [65535, 1], count_type="u16")
    with pytest.raises(oracle_mod.OracleError) as e:
        oracle_mod.bfs(sys, max_depth=2)
    assert e.value.status == oracle_mod.ERR_OVERFLOW


# --------------------------------------------------------------------------
# Deterministic branch (first applicable rule in every neuron): closed forms.
# --------------------------------------------------------------------------
def test_deterministic_closed_forms(oracle_mod):
    d = oracle_mod.deterministic(EX, 25)          # C_k = (2, 1, 1 + k): rules 1, 3, 4 forever
    assert d.final.tolist() == [2, 1, 26] and d.halt_step == -1 and d.first_repeat == -1 and d.steps_done == 25
    d = oracle_mod.deterministic(EX_TB, 25)       # C_1 = (2,1,2) is a fixed point (rules 1, 3, 5)
    assert d.final.tolist() == [2, 1, 2] and d.first_repeat == 2 and d.halt_step == -1
    d = oracle_mod.deterministic(EX_TB, 25, c0=[0, 1, 1])  # 011 -> 101 -> 100, which halts
    assert d.final.tolist() == [1, 0, 0] and d.halt_step == 2 and d.steps_done == 2


GAMMA = 0x9E3779B97F4A7C15


def test_config_hash_weights_are_splitmix64_stream(oracle_mod):
    # H of a unit vector e_n is the n-th output of SplitMix64 seeded with 0
    r = synth.SplitMix64(0)
    for n in range(5):
        e = [0] * 5
        e[n] = 1
        assert oracle_mod.config_hash(e) == r.next_u64()
    # linear in C (mod 2^64)
    a, b = [3, 0, 7, 1], [1, 2, 0, 5]
    s = [x + y for x, y in zip(a, b)]
    assert oracle_mod.config_hash(s) == (oracle_mod.config_hash(a) + oracle_mod.config_hash(b)) % (1 << 64)


def test_deterministic_digest_structure(oracle_mod):
    # digest = sum over computed steps k of mix64(H(C_k) + k * gamma)
    d0 = oracle_mod.deterministic(EX_TB, 0, c0=[1, 0, 0])
    assert d0.digest == oracle_mod.mix64(oracle_mod.config_hash([1, 0, 0])) and d0.steps_done == 0
    d1 = oracle_mod.deterministic(EX_TB, 1, c0=[0, 1, 1])   # C_1 = (1, 0, 1)
    want1 = (oracle_mod.mix64(oracle_mod.config_hash([0, 1, 1]))
             + oracle_mod.mix64(oracle_mod.config_hash([1, 0, 1]) + GAMMA)) % (1 << 64)
    assert d1.digest == want1


# --------------------------------------------------------------------------
# child_at: the child with index t equals row t of the full enumeration, for
# every t < Psi, on every configuration a walk reaches; index Psi is refused.
# --------------------------------------------------------------------------
def _child_at_cases():
    from tests.test_gpu_parity import twin_system

    cases = [("paper", EX, 12), ("textbook", EX_TB, 12), ("twins", twin_system(), 6)]
    cases += [(f"tiny{s}", synth.config_system(1, s), 6) for s in range(20)]
    return cases


@pytest.mark.parametrize("name,system,depth", _child_at_cases(), ids=lambda x: x if isinstance(x, str) else "")
def test_child_at_equals_enumeration(oracle_mod, name, system, depth):
    walk = oracle_mod.bfs(system, max_depth=depth, expand_max_count=9 if name == "paper" else -1)
    for C in walk.rows[:60]:
        rows, _, psi = oracle_mod.children(system, C, max_out=4096)
        assert psi <= 4096
        for t in range(psi):
            assert oracle_mod.child_at(system, C, t).tolist() == rows[t].tolist(), (name, C.tolist(), t)
        with pytest.raises(oracle_mod.OracleError):
            oracle_mod.child_at(system, C, psi)


def test_child_at_bruteforce_order(oracle_mod):
    """child_at against the brute-force order of the valid 0/1 spiking vectors
    (rule 1 most significant) with a dense C + S.M, on random tiny systems."""
    for seed in range(10):
        s = synth.config_system(1, seed)
        M = oracle_mod.matrix_dense(s)
        C = np.asarray(s.c0, dtype=np.int64)
        valid = [v for v in _valid_vectors_bruteforce(s, C)]
        for t, v in enumerate(valid):
            want = C + np.asarray(v, dtype=np.int64) @ M
            assert oracle_mod.child_at(s, C, t).tolist() == want.tolist()


def _valid_vectors_bruteforce(s, C):
    r = len(s.rule_i)
    for bits in range(2 ** r - 1, -1, -1):
        v = [(bits >> (r - 1 - k)) & 1 for k in range(r)]
        ok = True
        for n in range(s.m):
            ks = [k for k in range(r) if s.rule_neuron[k] == n]
            app = [k for k in ks if re.fullmatch(f"a{{{s.rule_i[k]}}}(?:a{{{s.rule_j[k]}}})*", "a" * int(C[n]))
                   and C[n] >= s.rule_c[k]]
            fired = [k for k in ks if v[k]]
            if any(k not in app for k in fired) or len(fired) != (1 if app else 0):
                ok = False
                break
        if ok:
            yield v


# --------------------------------------------------------------------------
# Deterministic walk: the breadth-first walk that keeps only the first spiking
# vector of every configuration is the single-branch trajectory, cut at its
# first repeat (empty frontier) or at its halting configuration.
# --------------------------------------------------------------------------
def _trajectory(oracle_mod, s, steps, c0=None):
    rows = [np.asarray(s.c0 if c0 is None else c0, dtype=np.int64)]
    for k in range(1, steps + 1):
        rows.append(oracle_mod.deterministic(s, k, c0=c0).final)
    return rows


def test_deterministic_walk_closed_forms(oracle_mod):
    w = oracle_mod.bfs(EX, max_depth=30, deterministic=True)     # C_k = (2, 1, 1 + k)
    assert w.level_sizes.tolist() == [1] * 31 and w.stop_reason == oracle_mod.STOP_DEPTH
    assert [r.tolist() for r in w.rows] == [[2, 1, 1 + k] for k in range(31)]
    assert w.tindex.tolist() == [-1] + [0] * 30
    w = oracle_mod.bfs(EX_TB, deterministic=True)                 # (2,1,1) -> (2,1,2), a fixed point
    assert [r.tolist() for r in w.rows] == [[2, 1, 1], [2, 1, 2]]
    assert w.stop_reason == oracle_mod.STOP_EMPTY_FRONTIER
    w = oracle_mod.bfs(EX_TB, c0=[0, 1, 1], deterministic=True)   # 011 -> 101 -> 100, halting
    assert [r.tolist() for r in w.rows] == [[0, 1, 1], [1, 0, 1], [1, 0, 0]]
    assert w.stop_reason == oracle_mod.STOP_ALL_HALTING


@pytest.mark.parametrize("seed", range(0, 40, 3))
def test_deterministic_walk_is_trajectory(oracle_mod, seed):
    s = synth.config_system(1, seed)
    d = oracle_mod.deterministic(s, 60)
    w = oracle_mod.bfs(s, deterministic=True, max_depth=60)
    traj = _trajectory(oracle_mod, s, d.steps_done)
    if d.first_repeat >= 0:
        n = d.first_repeat
        assert w.stop_reason == oracle_mod.STOP_EMPTY_FRONTIER
    elif d.halt_step >= 0:
        n = d.halt_step + 1
        assert w.stop_reason == oracle_mod.STOP_ALL_HALTING
    else:
        n = 61
        assert w.stop_reason == oracle_mod.STOP_DEPTH
    assert [r.tolist() for r in w.rows] == [r.tolist() for r in traj[:n]]


# ---------------------------------------------------------------------------
# The output neuron (Definition 1's out): the numbers a system generates are
# the steps between the first two spikes the output neuron sends to the
# environment (Section 2.1; the example generates N - {1}).
# ---------------------------------------------------------------------------
def test_example_generates_n_minus_one(oracle_mod):
    """Worked by hand under the textbook reading (E = a^k, rule 5 forgets two
    spikes): sigma_3 spikes at step 1; sigma_1 picks rule 1 (back to 2-1-2,
    sigma_3 forgetting) until it picks rule 2 at some step s >= 1, giving
    1-1-2, then 2-0-1, whose step s + 2 sends the second spike: s + 1 for
    every s >= 1, so the computations of at most D steps generate {2 .. D-1}."""
    tb = synth.paper_example(True)
    for D in range(1, 31):
        res = oracle_mod.bfs(tb, max_depth=D, out_neuron=3)
        assert oracle_mod.generated_numbers(res, 3) == list(range(2, D)), D
    # rows never carry an elapsed count before the first spike
    rows = oracle_mod.bfs(tb, max_depth=12, out_neuron=3).rows
    assert (rows[rows[:, 3] == 0, 4] == 0).all()


def _paths_generated(oracle_mod, s, out, depth):
    """Brute force over every computation of at most `depth` steps (no
    deduplication): the spike train of neuron `out` (1-based) along each path,
    and the gap between its first two spikes."""
    outs = [k for k in range(len(s.rule_neuron)) if int(s.rule_neuron[k]) == out - 1]
    found = set()

    def walk(C, d, times):
        if len(times) >= 2:
            found.add(times[1] - times[0])
            return
        if d == depth:
            return
        rows, S, psi = oracle_mod.children(s, C, max_out=4096)
        assert psi <= 4096
        for child, sv in zip(rows, S):
            q = sum(int(s.rule_p[k]) for k in outs if sv[k])
            walk(child, d + 1, times + [d + 1] * q)

    walk(np.asarray(s.c0, dtype=np.int64), 0, [])
    return sorted(found)


@pytest.mark.parametrize("seed", range(12))
def test_generated_numbers_match_all_paths(oracle_mod, seed):
    s = synth.config_system(1, seed)
    for out in (1, 2, 3):
        res = oracle_mod.bfs(s, max_depth=7, out_neuron=out)
        assert oracle_mod.generated_numbers(res, s.m) == _paths_generated(oracle_mod, s, out, 7), (seed, out)


def test_generated_numbers_of_the_example_match_all_paths(oracle_mod):
    for textbook in (True, False):
        s = synth.paper_example(textbook)
        res = oracle_mod.bfs(s, max_depth=9, out_neuron=3)
        assert oracle_mod.generated_numbers(res, 3) == _paths_generated(oracle_mod, s, 3, 9)
    # the simulator's reading of the rule file (at least k spikes) also generates 1:
    # sigma_3 may fire rule 4 again with 2 spikes right after its first spike
    res = oracle_mod.bfs(synth.paper_example(False), max_depth=6, out_neuron=3)
    assert oracle_mod.generated_numbers(res, 3)[0] == 1
