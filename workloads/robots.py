"""Seeded robot batches and load schedules (inputs only).

A robot is the cable-driven tube of Sec. II-A: a straight centreline of length
L split into n_e equal beam elements (Sec. II-B), clamped at a base that an
insertion stage pushes along the base direction, with three cables welded at
the distal end (Fig. 1b/c) whose tensions are the actuation inputs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


@dataclass
class RobotBatch:
    """A batch of independent robots sharing one section, material and lumen.

    Arrays are per robot (leading dimension B).  Units are SI.
    """
    n_elem: np.ndarray            # int32 [B]   number of beam elements
    length: np.ndarray            # f64   [B]   centreline length L
    base_pos: np.ndarray          # f64   [B,3] base node position before insertion
    base_dir: np.ndarray          # f64   [B,3] unit centreline direction at the base
    base_up: np.ndarray           # f64   [B,3] unit section axis y at the base (perp. to base_dir)
    tensions: np.ndarray          # f64   [B,n_cables] final cable tensions (N)
    depth: np.ndarray             # f64   [B]   final insertion depth (m)
    r_out: float = 1.5e-3
    r_in: float = 1.0e-3
    E: float = 50e6
    nu: float = 0.45
    cable_radius: float = 1.2e-3
    cable_angle: np.ndarray = field(default_factory=lambda: np.array([0.0, 2 * np.pi / 3, 4 * np.pi / 3]))
    contact_radius: float = 1.5e-3   # robot radius used as the contact offset r_c
    contact_margin: float = 1.0e-3   # detection band beyond r_c (delta)
    beta0: float = 1.0e-3            # step-size limit of the post-processing rule
    guide_len: float = 0.0           # straight insertion guide from the initial base (m)
    tip_len: float = 0.0             # distal bending section with the tube section above (m);
                                     # elements proximal to it use the shaft material below
    shaft_E: float = 510e6           # shaft: the robot row of the paper's material table
    shaft_A: float = 5.551e-6
    shaft_I: float = 5.041e-12
    n_load_steps: int = 20
    tension_ramp_steps: int = 20     # tensions reach their final value at this step
    depth_ramp_steps: int = 20       # insertion depth reaches its final value at this step

    @property
    def n_robots(self) -> int:
        return int(self.n_elem.shape[0])

    @property
    def n_nodes(self) -> np.ndarray:
        return self.n_elem.astype(np.int64) + 1

    @property
    def node_offset(self) -> np.ndarray:
        off = np.zeros(self.n_robots + 1, dtype=np.int64)
        off[1:] = np.cumsum(self.n_nodes)
        return off

    def subset(self, idx) -> "RobotBatch":
        idx = np.asarray(idx)
        kw = {k: getattr(self, k) for k in self.__dataclass_fields__}
        for k in ("n_elem", "length", "base_pos", "base_dir", "base_up", "tensions", "depth"):
            kw[k] = np.ascontiguousarray(getattr(self, k)[idx])
        return RobotBatch(**kw)


def load_schedule(rb: RobotBatch, k: int):
    """Depth and tensions applied at load step k (1-based): linear ramps."""
    ft = min(1.0, k / max(1, rb.tension_ramp_steps))
    fd = min(1.0, k / max(1, rb.depth_ramp_steps))
    return rb.depth * fd, rb.tensions * ft


def schedule_table(rb: RobotBatch, n_steps: int | None = None):
    """The load steps 1..n_steps of load_schedule as tables: tensions [n, B, n_cables]
    and depths [n, B] (the layout of an explicit load-step schedule)."""
    n = rb.n_load_steps if n_steps is None else n_steps
    steps = [load_schedule(rb, k) for k in range(1, n + 1)]
    return (np.ascontiguousarray(np.stack([t for _, t in steps])),
            np.ascontiguousarray(np.stack([d for d, _ in steps])))


def _frames(B, rng=None, roll=False):
    d = np.tile(np.array([0.0, 0.0, 1.0]), (B, 1))
    if roll and rng is not None:
        a = rng.uniform(0.0, 2 * np.pi, size=B)
        up = np.stack([np.cos(a), np.sin(a), np.zeros(B)], axis=1)
    else:
        up = np.tile(np.array([1.0, 0.0, 0.0]), (B, 1))
    return d, up


def robots_for_config(cfg: int, n_robots: int | None = None) -> RobotBatch:
    """Robot batch of configuration `cfg` (0..4), seeded with default_rng([cfg, 1])."""
    rng = np.random.default_rng([cfg, 1])
    if cfg == 0:
        B = 1
        d, up = _frames(B)
        return RobotBatch(
            n_elem=np.array([20], np.int32), length=np.array([0.30]),
            base_pos=np.zeros((B, 3)), base_dir=d, base_up=up,
            tensions=rng.uniform(0.0, 2.0, size=(B, 3)), depth=np.zeros(B),
            n_load_steps=20, tension_ramp_steps=20, depth_ramp_steps=20)
    if cfg in (1, 2):
        B = 1
        d, up = _frames(B)
        n_e = 200 if cfg == 1 else 1000
        depth = 0.30 if cfg == 1 else 0.30
        return RobotBatch(
            n_elem=np.array([n_e], np.int32), length=np.array([0.60]),
            base_pos=np.array([[0.0, 0.0, -0.60]]), base_dir=d, base_up=up,
            tensions=rng.uniform(0.0, 2.0, size=(B, 3)), depth=np.array([depth]),
            n_load_steps=100, tension_ramp_steps=10, depth_ramp_steps=100, guide_len=0.60, tip_len=0.07)
    if cfg == 3:
        B = 4096 if n_robots is None else n_robots
        n_e = rng.integers(50, 401, size=4096).astype(np.int32)[:B]
        T = rng.uniform(0.0, 3.0, size=(4096, 3))[:B]
        depth = rng.uniform(0.1, 0.5, size=4096)[:B]
        rad = 2e-3 * np.sqrt(rng.uniform(size=4096))[:B]
        ang = rng.uniform(0, 2 * np.pi, size=4096)[:B]
        d, up = _frames(B, rng, roll=True)
        bp = np.stack([rad * np.cos(ang), rad * np.sin(ang), np.full(B, -0.60)], axis=1)
        return RobotBatch(
            n_elem=n_e, length=np.full(B, 0.60), base_pos=bp, base_dir=d, base_up=up,
            tensions=T, depth=depth, n_load_steps=100, tension_ramp_steps=10,
            depth_ramp_steps=100, guide_len=0.60, tip_len=0.07)
    if cfg == 4:
        B = 1024 if n_robots is None else n_robots
        T = rng.uniform(0.0, 2.0, size=(1024, 3))[:B]
        depth = rng.uniform(0.1, 0.5, size=1024)[:B]
        rad = 2e-3 * np.sqrt(rng.uniform(size=1024))[:B]
        ang = rng.uniform(0, 2 * np.pi, size=1024)[:B]
        d, up = _frames(B, rng, roll=True)
        bp = np.stack([rad * np.cos(ang), rad * np.sin(ang), np.full(B, -0.60)], axis=1)
        return RobotBatch(
            n_elem=np.full(B, 300, np.int32), length=np.full(B, 0.60), base_pos=bp,
            base_dir=d, base_up=up, tensions=T, depth=depth, n_load_steps=100,
            tension_ramp_steps=10, depth_ramp_steps=100, guide_len=0.60, tip_len=0.07)
    raise ValueError(f"unknown configuration {cfg}")


# Sensor nodes of the differentiation workload: the nodes 0.0088 m and 0.0728 m from the tip,
# the offsets of the two distal sensor rows of the paper's material table (Table I), at the
# 2 mm element length of that workload (4 and 36 elements from the tip).
SENSOR_OFFSETS = (0.0088, 0.0728)


def sensor_nodes(rb: RobotBatch, b: int = 0):
    """Node indices counted from the tip (-1 = tip) of the sensors of robot b."""
    l0 = float(rb.length[b]) / int(rb.n_elem[b])
    return np.array([-1 - int(round(s / l0)) for s in SENSOR_OFFSETS], np.int32)


def sensor_targets(rb: RobotBatch, seed=(4, 2)):
    """Target positions [B, n_sensors, 3] of the sensors: their straight inserted positions
    (base position + (depth + arc length) along the base direction) plus N(0, 5 mm) per axis,
    seeded; defined from geometry only, without a solve."""
    rng = np.random.default_rng(list(seed))
    out = np.empty((rb.n_robots, len(SENSOR_OFFSETS), 3))
    for b in range(rb.n_robots):
        l0 = float(rb.length[b]) / int(rb.n_elem[b])
        n = int(rb.n_elem[b]) + 1
        for s, i in enumerate(sensor_nodes(rb, b)):
            arc = (n + int(i)) * l0
            out[b, s] = rb.base_pos[b] + (float(rb.depth[b]) + arc) * rb.base_dir[b]
    return out + rng.normal(scale=5e-3, size=out.shape)
