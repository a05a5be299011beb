"""Seeded generator of SN P systems without delays (Definition 1 of the paper).

A system is drawn as plain integers:

* rules, grouped by neuron in a total order (the paper orders rules neuron by
  neuron, Section 2.2), each with regular expression ``E = a^i (a^j)*``
  (``j = 0`` means exactly ``a^i``), consumption ``c`` and production ``p``;
* synapses ``(s, d)`` with ``s != d`` and no duplicates (Definition 1, item 3);
* the initial configuration ``C0`` (spikes per neuron, Section 2.2).

Random numbers come from SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), seeded with
``config_id << 32 | seed``.  Bounded integers are drawn by rejection, so every
value is exactly uniform.  The sampling order is fixed:

1. rule count of every neuron (config specific, see ``CONFIGS``);
2. for every neuron in order, for every one of its rules: ``i``, ``j``, ``c``, ``p``;
3. for every neuron in order: out-degree, then distinct targets ``!= self``
   drawn uniformly with rejection of repeats;
4. ``C0``, one count per neuron.

Nothing here evaluates the system: no matrix, no rule test, no step.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

_MASK64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


class SplitMix64:
    """SplitMix64 stream (Steele, Lea, Flood 2014): state advances by the golden gamma,
    output is the state passed through the variant-13 finaliser."""

    __slots__ = ("state",)

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + _GAMMA) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def below(self, n: int) -> int:
        """Uniform integer in [0, n) by rejection of the top partial block."""
        if n <= 0:
            raise ValueError("below() needs n >= 1")
        limit = ((1 << 64) // n) * n
        while True:
            x = self.next_u64()
            if x < limit:
                return x % n

    def uniform(self, lo: int, hi: int) -> int:
        """Uniform integer in the closed range [lo, hi]."""
        return lo + self.below(hi - lo + 1)

    def choice(self, values: Sequence[int]) -> int:
        return values[self.below(len(values))]


@dataclass
class System:
    """An SN P system as flat integer arrays (0-based neuron ids).

    ``count_type`` is ``"i32"`` or ``"u16"``: the element type the simulator
    stores spike counts in.
    """

    m: int
    rule_neuron: np.ndarray
    rule_i: np.ndarray
    rule_j: np.ndarray
    rule_c: np.ndarray
    rule_p: np.ndarray
    syn_src: np.ndarray
    syn_dst: np.ndarray
    c0: np.ndarray
    count_type: str = "i32"
    name: str = ""
    meta: dict = field(default_factory=dict)
    rule_d: Optional[np.ndarray] = None  # delay of every rule (None: a system without delays)

    @property
    def r(self) -> int:
        return int(self.rule_neuron.shape[0])

    @property
    def n_syn(self) -> int:
        return int(self.syn_src.shape[0])

    @property
    def count_max(self) -> int:
        return 65535 if self.count_type == "u16" else 2**31 - 1

    @property
    def np_dtype(self):
        return np.uint16 if self.count_type == "u16" else np.int32

    def rules(self) -> List[Tuple[int, int, int, int, int]]:
        return [
            (int(a), int(b), int(c), int(d), int(e))
            for a, b, c, d, e in zip(
                self.rule_neuron, self.rule_i, self.rule_j, self.rule_c, self.rule_p
            )
        ]


def _arr(values) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(values, dtype=np.int32))


def make_system(m, rules, syn, c0, count_type="i32", name="", meta=None) -> System:
    """Build a System from python lists: rules = [(neuron, i, j, c, p)] or
    [(neuron, i, j, c, p, d)] with a delay d, syn = [(s, d)]."""
    rules = list(rules)
    syn = list(syn)
    delays = any(len(x) > 5 for x in rules)
    return System(
        m=int(m),
        rule_neuron=_arr([x[0] for x in rules]),
        rule_i=_arr([x[1] for x in rules]),
        rule_j=_arr([x[2] for x in rules]),
        rule_c=_arr([x[3] for x in rules]),
        rule_p=_arr([x[4] for x in rules]),
        syn_src=_arr([s for s, _ in syn]),
        syn_dst=_arr([d for _, d in syn]),
        c0=np.ascontiguousarray(np.asarray(c0, dtype=np.int64)),
        count_type=count_type,
        name=name,
        meta=dict(meta or {}),
        rule_d=_arr([x[5] if len(x) > 5 else 0 for x in rules]) if delays else None,
    )


def with_delays(system: System, seed: int, d_max: int = 2, num: int = 1, den: int = 2) -> System:
    """Copy of ``system`` whose rules carry delays: for every rule in order, a
    draw below ``den`` that is below ``num`` gives it a delay uniform in
    [1, d_max], else 0 (stream seeded with ``6 << 32 | seed``)."""
    rng = SplitMix64(_seed(6, seed))
    d = []
    for _ in range(system.r):
        d.append(rng.uniform(1, d_max) if rng.below(den) < num else 0)
    return System(
        m=system.m, rule_neuron=system.rule_neuron, rule_i=system.rule_i, rule_j=system.rule_j,
        rule_c=system.rule_c, rule_p=system.rule_p, syn_src=system.syn_src, syn_dst=system.syn_dst,
        c0=system.c0, count_type=system.count_type, name=f"{system.name}_d{seed}",
        meta=dict(system.meta, delay_seed=seed, d_max=d_max), rule_d=_arr(d),
    )


def paper_example(textbook: bool = False) -> System:
    """The paper's 3-neuron system that generates N - {1} (Section 2.1, Figure 1),
    with C0 = <2, 1, 1> (Section 2.2) and synapses {(1,2),(1,3),(2,1),(2,3)}.

    Rule exponents come from the simulator's rule file ``2 2 $ 1 $ 1 2``
    (Section 4) and consumptions from the printed matrix M (Section 2.2):
    rule 1 consumes 1, rule 2 consumes 2, rule 3 consumes 1, rule 4 consumes 1,
    rule 5 consumes 2; rules 1-3 send one spike along each synapse, rules 4-5
    have no synapse (neuron 3 only emits to the environment).

    ``textbook=False`` reads an exponent k as ``E = a^k a*`` (the neuron needs at
    least k spikes): the reading under which the printed run of Section 5 is
    reproduced.  ``textbook=True`` reads it as ``E = a^k`` exactly (rule form b-3).
    """
    j = 0 if textbook else 1
    rules = [
        (0, 2, j, 1, 1),
        (0, 2, j, 2, 1),
        (1, 1, j, 1, 1),
        (2, 1, j, 1, 1),
        (2, 2, j, 2, 0),
    ]
    syn = [(0, 1), (0, 2), (1, 0), (1, 2)]
    return make_system(3, rules, syn, [2, 1, 1], name="paper_example_textbook" if textbook else "paper_example")


def random_system(
    rng: SplitMix64,
    m: int,
    rule_counts: Sequence[int],
    i_range: Tuple[int, int],
    j_values: Sequence[int],
    p_values: Sequence[int],
    outdeg: Tuple[int, int],
    c0_range: Tuple[int, int],
    count_type: str = "i32",
    name: str = "",
    meta: Optional[dict] = None,
) -> System:
    """Draw rules, synapses and C0 in the fixed sampling order (module docstring).

    ``c`` is uniform in [1, i]; ``j`` and ``p`` are uniform over the listed values.
    The out-degree is uniform in ``outdeg`` and clipped to ``m - 1``.
    """
    rules = []
    for n in range(m):
        for _ in range(rule_counts[n]):
            i = rng.uniform(i_range[0], i_range[1])
            j = rng.choice(j_values)
            c = rng.uniform(1, i)
            p = rng.choice(p_values)
            rules.append((n, i, j, c, p))
    syn = []
    for n in range(m):
        k = min(rng.uniform(outdeg[0], outdeg[1]), m - 1)
        chosen = []
        seen = set()
        while len(chosen) < k:
            d = rng.below(m)
            if d == n or d in seen:
                continue
            seen.add(d)
            chosen.append(d)
        syn.extend((n, d) for d in chosen)
    c0 = [rng.uniform(c0_range[0], c0_range[1]) for _ in range(m)]
    return make_system(m, rules, syn, c0, count_type=count_type, name=name, meta=meta)


# Configuration recipes.  Values follow the workload table of the build plan;
# the paper itself only runs its 3-neuron example (Section 5).
CONFIGS = {
    1: dict(name="tiny_plain", m=3, i=(1, 3), j=(0, 1, 2), p=(0, 1), outdeg=(2, 2), c0=(0, 3), count_type="i32"),
    2: dict(name="plain_sparse", m=64, rules=2, i=(1, 4), j=(0, 1, 2, 3), p=(0, 1), outdeg=(4, 4), c0=(0, 4), count_type="i32"),
    3: dict(name="dense_int8", m=512, rules=3, i=(1, 4), j=(0, 1, 2, 3), p=(0, 1, 2, 3, 4), outdeg=(64, 64), c0=(0, 4), count_type="i32"),
    4: dict(name="batched_uneven", m=(16, 1024), rules=(1, 3), i=(1, 4), j=(0, 1, 2, 3), p=(0, 1), outdeg=(2, 32), c0=(0, 4), count_type="i32"),
    5: dict(name="large_exploration", m=4096, rules=4, i=(1, 4), j=(0, 1, 2, 3), p=(0, 1), outdeg=(16, 16), c0=(0, 8), count_type="u16"),
}


def _seed(config_id: int, seed: int) -> int:
    return ((config_id & 0xFFFFFFFF) << 32) | (seed & 0xFFFFFFFF)


def config_system(config_id: int, seed: int = 0, m: Optional[int] = None) -> System:
    """System ``seed`` of configuration ``config_id`` (1, 2, 3 or 5; 4 is per system).

    ``m`` overrides the neuron count (used to build scaled-down cases of a
    recipe for tests); everything else stays the recipe's.
    """
    cfg = CONFIGS[config_id]
    rng = SplitMix64(_seed(config_id, seed))
    if config_id == 1:
        mm = cfg["m"] if m is None else m
        counts = [1] * mm
        for _ in range(2):  # two extra rules on uniform neurons: r = m + 2
            counts[rng.below(mm)] += 1
    elif config_id == 4:
        return batched_systems(seed, 1)[0] if m is None else _batched_one(seed, m)
    else:
        mm = cfg["m"] if m is None else m
        counts = [cfg["rules"]] * mm
    return random_system(
        rng, mm, counts, cfg["i"], cfg["j"], cfg["p"], cfg["outdeg"], cfg["c0"],
        count_type=cfg["count_type"], name=f"{cfg['name']}_s{seed}",
        meta=dict(config=config_id, seed=seed),
    )


def _batched_one(seed: int, m_fixed: Optional[int] = None) -> System:
    cfg = CONFIGS[4]
    rng = SplitMix64(_seed(4, seed))
    m = rng.uniform(cfg["m"][0], cfg["m"][1])
    if m_fixed is not None:
        m = m_fixed
    counts = [rng.uniform(cfg["rules"][0], cfg["rules"][1]) for _ in range(m)]
    return random_system(
        rng, m, counts, cfg["i"], cfg["j"], cfg["p"], cfg["outdeg"], cfg["c0"],
        count_type=cfg["count_type"], name=f"batched_s{seed}", meta=dict(config=4, seed=seed),
    )


def batched_systems(first_seed: int = 0, count: int = 256) -> List[System]:
    """Systems ``first_seed .. first_seed + count - 1`` of the batched recipe:
    m uniform in [16, 1024], then per neuron 1-3 rules, out-degree in [2, 32]."""
    return [_batched_one(first_seed + k) for k in range(count)]
