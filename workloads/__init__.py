"""Seeded synthetic inputs for the eikonal solver and its checks.

This module only *generates* inputs (speed fields, source sets, receiver sets,
adjoint seeds). It holds none of the solver's arithmetic, so both the GPU path
and the CPU oracle can consume the same arrays without sharing method code.
"""

from .gen import (  # noqa: F401
    BASE_SEED,
    Problem,
    lognormal_field,
    maze_field,
    layered_anomaly_field,
    tiny_constant,
    lognormal_2d,
    maze_3d,
    layered_3d,
    batch_2d,
    random_problem,
    receivers_on_face,
    flat_index,
    paper_example,
    PAPER_SIZES,
)
