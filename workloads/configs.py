"""The five workload configurations (robots + lumen + schedule)."""
from __future__ import annotations

import os
import numpy as np

from .robots import robots_for_config
from .lumen import lumen_for_config

CONFIGS = {
    0: "plain-fp64 single: 20 elements, L=0.30 m, straight 512-triangle cylinder, tension ramp",
    1: "plain-fp64 realistic: 200 elements, L=0.60 m, 3-level branching lumen (50k tri), 100 insertion steps",
    2: "mixed: 1000 elements, L=0.60 m, 5-level branching lumen (200k tri), 100 insertion steps",
    3: "batched: 4096 robots, 50..400 elements, L=0.60 m, shared 50k-triangle lumen, 100 steps",
    4: "differentiation: 1024 robots x 300 elements, shared 50k-triangle lumen, tip-sensor loss",
}

_CACHE_DIR = os.environ.get("ACCFEM_MESH_CACHE", os.path.join(os.path.dirname(__file__), ".cache"))


def _cached_lumen(cfg):
    key = {0: 0, 1: 1, 3: 1, 4: 1, 2: 2}[cfg]
    path = os.path.join(_CACHE_DIR, f"lumen_{key}.npz")
    if os.path.exists(path):
        z = np.load(path)
        return z["verts"], z["tris"]
    V, T = lumen_for_config(key)
    try:
        os.makedirs(_CACHE_DIR, exist_ok=True)
        np.savez(path, verts=V, tris=T)
    except OSError:
        pass
    return V, T


def make_config(cfg: int, n_robots: int | None = None):
    """Return (RobotBatch, verts, tris) of configuration `cfg`."""
    rb = robots_for_config(cfg, n_robots)
    V, T = _cached_lumen(cfg)
    return rb, V, T
