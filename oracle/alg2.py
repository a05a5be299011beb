"""Algorithm 2 (Section 4.2) with the paper's own Python-list representation.

TEST INFRASTRUCTURE ONLY (part of the oracle).  It restates steps II-1, II-2
and II-3 on lists of strings so that the worked example's intermediate lists
``tmp``, ``tmp2`` and ``tmp3`` can be compared with the values the paper
prints, and so that the C oracle's enumeration order can be checked against
this independent formulation on small systems.

Readings (the paper is silent on them):
* rule applicability is passed in as a predicate, so both readings of the
  exponent in the rule file (exactly ``a^k`` or at least ``k`` spikes) can be
  exercised;
* a neuron with no applicable rule contributes the all-zero string (it fires
  nothing), i.e. factor 1 in the product Psi rather than 0.
"""
from __future__ import annotations

from typing import Callable, List, Sequence


def step_ii1(conf: Sequence[int], rules: Sequence[Sequence[object]],
             applies: Callable[[int, object], bool]) -> List[List[int]]:
    """II-1: copy r into tmp, numbering the rules of each neuron that satisfy E
    as 1, 2, ... in order and marking the others 0."""
    tmp = []
    for n, neuron_rules in enumerate(rules):
        marks, count = [], 0
        for rule in neuron_rules:
            if applies(conf[n], rule):
                count += 1
                marks.append(count)
            else:
                marks.append(0)
        tmp.append(marks)
    return tmp


def omega(tmp_neuron: Sequence[int]) -> int:
    """omega: the largest mark of a neuron, i.e. how many of its rules apply."""
    return max(tmp_neuron) if tmp_neuron else 0


def step_ii2(tmp: Sequence[Sequence[int]]) -> List[List[str]]:
    """II-2: per neuron, one string per applicable rule with a 1 in that rule's
    position and 0 elsewhere; all zeros when no rule of the neuron applies."""
    tmp2 = []
    for marks in tmp:
        strings = []
        for want in range(1, omega(marks) + 1):
            strings.append("".join("1" if x == want else "0" for x in marks))
        if not strings:
            strings.append("0" * len(marks))
        tmp2.append(strings)
    return tmp2


def step_ii3(tmp2: Sequence[Sequence[str]]) -> List[str]:
    """II-3: pair the neurons in order, distributing every string gathered so far
    over every string of the next neuron (m - 1 pairings)."""
    tmp3 = list(tmp2[0])
    for nxt in tmp2[1:]:
        tmp3 = [a + b for a in tmp3 for b in nxt]
    return tmp3


def psi(tmp: Sequence[Sequence[int]]) -> int:
    """Psi = product over neurons of the number of applicable rules (each neuron
    with none counted as 1, see the module docstring)."""
    out = 1
    for marks in tmp:
        out *= max(1, omega(marks))
    return out


def spiking_vectors(conf, rules, applies):
    """All valid spiking vectors of ``conf`` as strings, in II-3 order."""
    return step_ii3(step_ii2(step_ii1(conf, rules, applies)))
