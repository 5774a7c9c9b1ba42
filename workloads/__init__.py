"""Seeded synthetic inputs shared by the oracle, the GPU path's tests and the bench.

This package synthesises *inputs only*: robot discretisations, cable tensions,
insertion schedules and triangulated lumen meshes shaped like the paper's
workloads (Sec. II-A robot, Sec. II-C MRI-reconstructed cavity mesh, Sec. IV
bronchial insertion).  It contains none of the method's arithmetic (no element
forces, no collision predicate, no solver), so that the oracle and the HIP path
can both consume it without sharing any of the computation under test.
"""
from .robots import (RobotBatch, robots_for_config, load_schedule, schedule_table, sensor_nodes,
                     sensor_targets)
from .lumen import straight_cylinder_mesh, branching_lumen_mesh, lumen_for_config
from .configs import CONFIGS, make_config

__all__ = [
    "RobotBatch", "robots_for_config", "load_schedule", "schedule_table", "sensor_nodes",
    "sensor_targets",
    "straight_cylinder_mesh", "branching_lumen_mesh", "lumen_for_config",
    "CONFIGS", "make_config",
]
