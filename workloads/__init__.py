"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package only draws particle distributions (positions, velocities,
masses, times, active sets).  It contains none of the force arithmetic:
no pair interaction, no potential, no predictor.  Both the CPU oracle tests
and the GPU path take their inputs from here so that they see identical
arrays; neither side's results ever flow back into these generators.
"""

from .generators import (  # noqa: F401
    plummer,
    salpeter_masses,
    hard_binaries,
    synthetic_derivatives,
    JMemory,
    make_jmemory,
    config_c1,
    config_c2,
    config_c3,
    config_c5,
    config_c4,
    ClusterBatch,
    active_set,
    random_cluster,
    input_digest,
)
