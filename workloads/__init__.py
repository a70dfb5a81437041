"""Seeded synthetic workloads: QAOA circuit descriptions for noisy neutral-atom chains.

This package only draws numbers (chain length, levels, depth, angles, noise rates,
bond-dimension cap) from a seeded generator.  It holds none of the simulation's
arithmetic: no matrices, no channels, no tensors.  Both the CPU oracle (in tests)
and the GPU library's drivers read the same descriptions from here.
"""
from .qaoa import (  # noqa: F401
    CircuitSpec,
    config_m0,
    config_m1,
    config_m2_batch,
    config_m3,
    noiseless_spec,
    random_spec,
)
