"""Seeded synthetic workloads for the bidomain per-step solve.

This package only generates inputs: meshes, region tags, fibre frames,
conductivity values, stimulus masks and run lengths.  It holds none of the
method's arithmetic (no assembly, no time stepping, no solver), so that the
CPU oracle and the HIP path can both consume it without sharing any code.
"""
from .meshes import (  # noqa: F401
    REGION_TORSO, REGION_HEART, REGION_LUNG,
    square2d, thorax2d, slab3d, make_config, config_names,
    summary,
)
