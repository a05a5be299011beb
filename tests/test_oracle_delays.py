"""Pins of the oracle's step for SN P systems with delays.

The paper simulates systems without delays and leaves the variant with delays
to the work it cites (Section 2.1, opening).  The oracle takes that variant's
usual definition: a rule with delay d >= 1 used at step s takes its spikes at
once, its neuron is closed at steps s .. s+d-1 (it fires nothing and loses the
spikes sent to it), sends its spikes at step s+d (keeping what it receives
then, firing nothing), and fires again from step s+d+1.  A row holds the
counts, then (wait, pend) of every neuron owning a rule with a delay.

Pinned here, on the CPU, against things other than the oracle's own code:
  * hand-worked runs of small systems, each derived step by step below from
    the definition (lost spikes, the sending step, nondeterministic delays,
    a number generated through the output neuron);
  * every delay 0: the step must reduce to C' = C + S.M, so walks equal the
    delay-free walks (which are pinned to the paper's printed run);
  * a brute force on tiny random systems: every path of every length written
    with send times and closed intervals instead of countdowns; BFS levels
    with global deduplication are the distance layers of the reachable set.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from synth.systems import make_system, with_delays


def rows_of(res):
    return [tuple(int(x) for x in r) for r in res.rows]


# ---------------------------------------------------------------------------
# Hand-worked runs.  Neurons are 0-based; rules (neuron, i, j, c, p, d) with
# E = a^i (a^j)* (j = 0: exactly a^i).  Row = counts, then (wait, pend) of the
# delayed neurons in neuron order.
# ---------------------------------------------------------------------------
def test_chain_with_a_delay():
    # n0: a -> a; 2, synapse n0 -> n1; n1: a -> a; 0, synapse n1 -> n2; n2 no rule.
    # step 0: n0 fires, takes its spike, waits 2 (sends nothing) -> (0,0,0 | 2,1)
    # step 1: n0 closed (wait 2 -> 1)                           -> (0,0,0 | 1,1)
    # step 2: n0 sends 1 to n1 (wait 1 -> 0)                    -> (0,1,0 | 0,0)
    # step 3: n1 fires, sends 1 to n2                           -> (0,0,1 | 0,0)
    # step 4: nothing applies and nobody waits: halting.
    s = make_system(3, [(0, 1, 0, 1, 1, 2), (1, 1, 0, 1, 1, 0)], [(0, 1), (1, 2)], [1, 0, 0])
    assert oracle.row_width(s) == 5
    res = oracle.bfs(s)
    assert rows_of(res) == [(1, 0, 0, 0, 0), (0, 0, 0, 2, 1), (0, 0, 0, 1, 1), (0, 1, 0, 0, 0), (0, 0, 1, 0, 0)]
    assert res.level_sizes.tolist() == [1, 1, 1, 1, 1]
    assert res.stop_reason == oracle.STOP_ALL_HALTING
    # a parent with nothing applicable but a neuron waiting is not halting
    assert res.halting.tolist() == [0, 0, 0, 0, 1]
    assert res.enumerated.tolist() == [1, 1, 1, 1, 0]


def test_spike_sent_to_a_closed_neuron_is_lost():
    # n0: a -> a; 0, synapse n0 -> n1.  n1: a -> a; 1, synapse n1 -> n2.  n2 no rule.
    # step 0: n0 sends 1 to n1, but n1 fires its delayed rule at this step, so it
    #         is closed and the spike is lost                  -> (0,0,0 | 1,1)
    # step 1: n1 sends 1 to n2                                  -> (0,0,1 | 0,0)
    s = make_system(3, [(0, 1, 0, 1, 1, 0), (1, 1, 0, 1, 1, 1)], [(0, 1), (1, 2)], [1, 1, 0])
    res = oracle.bfs(s)
    assert rows_of(res) == [(1, 1, 0, 0, 0), (0, 0, 0, 1, 1), (0, 0, 1, 0, 0)]
    assert res.stop_reason == oracle.STOP_ALL_HALTING


def test_neuron_receives_at_its_sending_step():
    # n0: E = a(a)*, c 1, p 1, d 0, synapse n0 -> n1.  n1: a -> a; 1, synapse n1 -> n2.
    # step 0: n0 (2 spikes) sends 1; n1 fires its delayed rule, closed: lost
    #                                                           -> (1,0,0 | 1,1)
    # step 1: n0 sends 1; n1 sends its pending spike to n2 and is open at this
    #         step, so it keeps n0's spike                      -> (0,1,1 | 0,0)
    # step 2: n1 fires again                                    -> (0,0,1 | 1,1)
    # step 3: n1 sends                                          -> (0,0,2 | 0,0)
    s = make_system(3, [(0, 1, 1, 1, 1, 0), (1, 1, 0, 1, 1, 1)], [(0, 1), (1, 2)], [2, 1, 0])
    res = oracle.bfs(s)
    assert rows_of(res) == [(2, 1, 0, 0, 0), (1, 0, 0, 1, 1), (0, 1, 1, 0, 0), (0, 0, 1, 1, 1), (0, 0, 2, 0, 0)]


def test_no_rule_fires_at_the_sending_step():
    # n0: E = a(a)*, c 1, p 1, d 1, synapse n0 -> n1; n1 no rule.
    # step 0: n0 (2 spikes) fires                              -> (1,0 | 1,1)
    # step 1: n0 sends; it holds a spike its rule could take, but it fires
    #         nothing at the step it sends                     -> (1,1 | 0,0)
    # step 2: n0 fires                                          -> (0,1 | 1,1)
    # step 3: n0 sends                                          -> (0,2 | 0,0)
    s = make_system(2, [(0, 1, 1, 1, 1, 1)], [(0, 1)], [2, 0])
    res = oracle.bfs(s)
    assert rows_of(res) == [(2, 0, 0, 0), (1, 0, 1, 1), (1, 1, 0, 0), (0, 1, 1, 1), (0, 2, 0, 0)]


def test_rules_that_differ_only_in_delay_are_distinct_choices():
    # n0 holds 1 spike with a -> a; 0 and a -> a; 1 (same c and p), synapse n0 -> n1.
    # children of C0 in Algorithm 2 order: the first rule (0,1 | 0,0), the second
    # (0,0 | 1,1).  The second's child sends at the next step: (0,1 | 0,0) again,
    # a repeat, so the walk ends with an empty frontier.
    s = make_system(2, [(0, 1, 0, 1, 1, 0), (0, 1, 0, 1, 1, 1)], [(0, 1)], [1, 0])
    res = oracle.bfs(s)
    assert rows_of(res) == [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 1)]
    assert res.tindex.tolist() == [-1, 0, 1]
    assert res.level_sizes.tolist() == [1, 2]
    assert res.enumerated.tolist() == [2, 1]
    assert res.halting.tolist() == [0, 1]
    assert res.stop_reason == oracle.STOP_EMPTY_FRONTIER


@pytest.mark.parametrize("delays", [(2,), (2, 4), (1, 3, 5)])
def test_output_neuron_generates_the_delays(delays):
    # n0 holds 1 spike with a -> a; 0 and a -> a; d for every d listed, synapse
    # n0 -> n2.  n1 holds 1 spike with a -> a; 0, synapse n1 -> n2.  n2 (output)
    # sends one spike to the environment with a -> a (and a^2 -> a, c 2).
    # With a delayed rule d: step 0 n1 sends to n2; step 1 n2 fires (first spike
    # out); n0 sends at step d, n2 fires at step d + 1: the second spike comes
    # d steps after the first.  With n0's delay-0 rule both spikes reach n2 at
    # step 0, it fires a^2 once: one spike out, no number.  So the system
    # generates exactly the listed delays.
    rules = [(0, 1, 0, 1, 1, 0)] + [(0, 1, 0, 1, 1, d) for d in delays]
    rules += [(1, 1, 0, 1, 1, 0), (2, 1, 0, 1, 1, 0), (2, 2, 0, 2, 1, 0)]
    s = make_system(3, rules, [(0, 2), (1, 2)], [1, 1, 0])
    res = oracle.bfs(s, out_neuron=3, max_depth=2 * max(delays) + 6)
    assert oracle.generated_numbers(res, 3) == sorted(delays)


# ---------------------------------------------------------------------------
# Every delay 0: the same walk as the system without delays.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(12))
def test_zero_delays_reduce_to_the_plain_step(seed):
    s = synth.config_system(1, seed)
    z = with_delays(s, seed, num=0)
    assert z.rule_d is not None and not z.rule_d.any()
    kw = [dict(max_depth=8), dict(max_depth=8, out_neuron=1 + seed % 3), dict(max_depth=8, frontier_cap=3),
          dict(max_depth=8, child_budget=5), dict(max_depth=8, expand_max_count=3)]
    for k in kw:
        a, b = oracle.bfs(s, **k), oracle.bfs(z, **k)
        assert a.rows.tolist() == b.rows.tolist(), k
        assert a.level_sizes.tolist() == b.level_sizes.tolist()
        assert a.parent.tolist() == b.parent.tolist() and a.tindex.tolist() == b.tindex.tolist()
        assert a.enumerated.tolist() == b.enumerated.tolist() and a.halting.tolist() == b.halting.tolist()
        assert a.stop_reason == b.stop_reason


def test_zero_delay_plain_sparse_system():
    s = synth.config_system(2, 1, m=12)
    z = with_delays(s, 3, num=0)
    a, b = oracle.bfs(s, max_depth=4), oracle.bfs(z, max_depth=4)
    assert a.rows.tolist() == b.rows.tolist() and a.enumerated.tolist() == b.enumerated.tolist()


# ---------------------------------------------------------------------------
# Brute force: send times and closed intervals.
# ---------------------------------------------------------------------------
def _brute_children(s, row):
    """Every child of `row` (time re-based to step 0), written with absolute
    send times: a delayed neuron waiting w >= 1 sends at step w - 1 and is
    closed on [0, w - 2]; firing a rule with delay d >= 1 at step 0 closes it
    on [0, d - 1] and makes it send at step d."""
    m = s.m
    delayed = [n for n in range(m) if any(int(s.rule_d[k]) > 0 and int(s.rule_neuron[k]) == n for k in range(s.r))]
    col = {n: m + 2 * q for q, n in enumerate(delayed)}
    counts = list(row[:m])
    send_at = {n: row[col[n]] - 1 for n in delayed if row[col[n]] >= 1}   # absolute send step
    amount = {n: row[col[n] + 1] for n in send_at}
    choices = []
    for n in range(m):
        if n in send_at:                 # busy from its firing step up to its send step
            choices.append([None])
            continue
        app = []
        for k in range(s.r):
            if int(s.rule_neuron[k]) != n:
                continue
            i, j, c = int(s.rule_i[k]), int(s.rule_j[k]), int(s.rule_c[k])
            x = counts[n]
            ok = x >= c and x >= i and ((x - i) % j == 0 if j else x == i)
            if ok:
                app.append(k)
        choices.append(app if app else [None])
    if not any(ch != [None] for ch in choices) and not send_at:
        return []
    kids = []
    for pick in itertools.product(*choices):
        closed_until = {n: send_at[n] - 1 for n in send_at}       # closed on [0, this]
        sends_now = {n: amount[n] for n in send_at if send_at[n] == 0}
        new_send, new_amt = {n: send_at[n] for n in send_at if send_at[n] >= 1}, {}
        for n in new_send:
            new_amt[n] = amount[n]
        nc = list(counts)
        for n, k in enumerate(pick):
            if k is None:
                continue
            nc[n] -= int(s.rule_c[k])
            d = int(s.rule_d[k])
            if d == 0:
                sends_now[n] = int(s.rule_p[k])
            else:
                closed_until[n] = d - 1
                new_send[n] = d
                new_amt[n] = int(s.rule_p[k])
        for e in range(s.n_syn):
            a, b = int(s.syn_src[e]), int(s.syn_dst[e])
            if a in sends_now and not (b in closed_until and closed_until[b] >= 0):
                nc[b] += sends_now[a]
        # the row one step later (time 1): a send step t >= 1 is t steps ahead
        tail = []
        for n in delayed:
            if n in new_send and new_send[n] >= 1:
                tail += [new_send[n], new_amt[n]]
            else:
                tail += [0, 0]
        kids.append(tuple(nc) + tuple(tail))
    return kids


def _brute_layers(s, c0, depth):
    seen = {c0}
    layers = [{c0}]
    for _ in range(depth):
        nxt = set()
        for row in layers[-1]:
            for ch in _brute_children(s, row):
                if ch not in seen:
                    nxt.add(ch)
        if not nxt:
            break
        seen |= nxt
        layers.append(nxt)
    return layers


@pytest.mark.parametrize("seed", range(16))
def test_walk_levels_are_the_brute_force_distance_layers(seed):
    base = synth.config_system(1, seed) if seed % 2 == 0 else synth.config_system(2, seed, m=5)
    s = with_delays(base, seed, d_max=1 + seed % 3)
    w = oracle.row_width(s)
    c0 = tuple(int(x) for x in s.c0) + (0,) * (w - s.m)
    depth = 7 if s.m <= 3 else 5
    layers = _brute_layers(s, c0, depth)
    res = oracle.bfs(s, max_depth=depth)
    got = [set(map(tuple, res.level(k).tolist())) for k in range(res.n_levels)]
    assert [len(x) for x in got] == res.level_sizes.tolist()  # no repeats inside a level
    assert got == layers[: len(got)]
    assert len(got) == len(layers)


def test_brute_force_sees_a_planted_mistake():
    """The brute force is strict enough to catch a wrong step: a copy of a
    system whose delayed rule keeps the spikes it is sent while closed would
    walk differently (planted on the CPU, in the expected side only)."""
    s = make_system(3, [(0, 1, 0, 1, 1, 0), (1, 1, 0, 1, 1, 1)], [(0, 1), (1, 2)], [1, 1, 0])
    layers = _brute_layers(s, (1, 1, 0, 0, 0), 4)
    wrong = [{(1, 1, 0, 0, 0)}, {(0, 1, 0, 1, 1)}]  # n1 keeping n0's spike while closed
    assert layers[:2] != wrong
    assert layers[1] == {(0, 0, 0, 1, 1)}


def test_delay_helpers_refuse_rows_with_states():
    s = make_system(2, [(0, 1, 0, 1, 1, 1)], [(0, 1)], [1, 0])
    with pytest.raises(oracle.OracleError):
        oracle.children(s, [1, 0])
    with pytest.raises(oracle.OracleError):
        oracle.deterministic(s, 3)


def test_row_width_counts_delayed_neurons():
    s = make_system(4, [(0, 1, 0, 1, 1, 0), (1, 1, 0, 1, 1, 3), (1, 2, 0, 1, 1, 0), (3, 1, 0, 1, 0, 2)],
                    [(0, 1)], [1, 0, 0, 0])
    assert oracle.row_width(s) == 4 + 2 * 2
    assert oracle.row_width(s, out_neuron=1) == 4 + 2 + 2 * 2
    z = make_system(2, [(0, 1, 0, 1, 1)], [(0, 1)], [1, 0])
    assert oracle.row_width(z) == 2
