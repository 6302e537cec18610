"""Seeded synthetic Join-Project inputs.

This module only draws input tables; it holds none of the Join-Project
arithmetic.  Both the CPU oracle and the GPU path consume what it produces.
"""
from .generators import (  # noqa: F401
    SEED_ROOT,
    Instance,
    zipf_sample,
    distinct_pairs,
    uniform_table,
    config1,
    config2,
    config3,
    config4,
    config5_trace,
    uniform_paper_default,
    zipf_xz_paper,
    small_random,
    config4_instance,
)
