"""Seeded synthetic workloads for the distance-threshold search.

This package only draws input geometry (segment endpoints, times, trajectory
ids and per-query thresholds). It holds none of the search's arithmetic: no
velocities, no distances, no overlaps. Both the oracle and the GPU library
consume its arrays.
"""
from .workloads import (  # noqa: F401
    Segments,
    CONFIGS,
    make_db,
    make_queries,
    make_config,
    seed_for,
    concat,
)
from . import fixtures  # noqa: F401
