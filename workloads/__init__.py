"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This package generates *data only*: scene geometry, a G-buffer, light and
occluder lists, and initial parameters.  It contains none of the cache's
arithmetic (no encoding, network, sampling, labelling or training step), so
both sides of every parity check can consume its arrays without sharing any
method code.
"""
from .configs import GridCfg, MlpCfg, Workload, WORKLOADS, get_workload
from .scenes import (
    unit_cube_scene,
    box_scene,
    init_params,
    pos_to_unit,
    moving_light,
    moving_light_table,
    LightAnimation,
)

__all__ = [
    "GridCfg", "MlpCfg", "Workload", "WORKLOADS", "get_workload",
    "unit_cube_scene", "box_scene", "init_params", "pos_to_unit", "moving_light",
    "moving_light_table", "LightAnimation",
]
