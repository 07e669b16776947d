"""Seeded synthetic inputs for the AMBER z_re hot path.

This module serves both the oracle tests and the GPU path.  It holds none of
the method's arithmetic: it only draws density, source and intensity fields
with the structure of the paper's workloads (see ``synth.py``).
"""
from .synth import (  # noqa: F401
    C3_HISTORIES,
    C3_LMFP,
    CONFIGS,
    BoxConfig,
    c4_boxes,
    c5_requests,
    config_seed,
    make_box,
    make_density,
    make_halos,
    make_intensity,
    make_weights_edge,
)
