"""Seeded synthetic SN P systems shared by the oracle tests, the GPU tests and the bench.

This package only draws numbers: rules ``(neuron, i, j, c, p)``, synapses and the
initial configuration.  It holds none of the simulation arithmetic (no matrix,
no applicability test, no enumeration), so the CPU oracle and the GPU path stay
independent of each other.
"""
from .systems import (  # noqa: F401
    SplitMix64,
    System,
    make_system,
    paper_example,
    random_system,
    config_system,
    batched_systems,
    CONFIGS,
)
