"""torch.autograd wrapper: sensor positions at equilibrium as a function of the cable tensions.

forward runs the load-stepped Newton solve of the HIP library and returns the
positions of the sensor nodes; backward calls fem_grad (the adjoint at the
converged state).  Tensors cross the boundary as host arrays (marshalling only).
"""
from __future__ import annotations

import numpy as np
import torch

from .fem import FEM_ACT_CABLES


class FEMEquilibrium(torch.autograd.Function):
    """apply(tensions [B, n_cables], ctx, sensor_nodes, depth [B] or None, n_load_steps,
    start_state [n_nodes, 7] or None) -> sensor positions [B, n_sensors, 3] (float64).

    The solve ramps from the context's last actuation to `tensions` over n_load_steps;
    with start_state it restarts from that state and ramps from zero tension.  The context must not be solved again or reset
    between forward and backward: backward checks this and raises otherwise.
    """

    @staticmethod
    def forward(ctx, tensions, fem_ctx, sensor_nodes, depth, n_load_steps, start_state):
        T = tensions.detach().to("cpu", torch.float64).contiguous().numpy()
        if start_state is not None:
            # the ramp starts at zero tension, at the target depth, from start_state
            fem_ctx.fem_set_state(start_state)
            fem_ctx.fem_set_actuation(FEM_ACT_CABLES, np.zeros(T.size), depth)
            fem_ctx.fem_solve(0, state=False, info=False)
        fem_ctx.fem_set_actuation(FEM_ACT_CABLES, T.ravel(), depth)
        out = fem_ctx.fem_solve(int(n_load_steps), state=True, info=False)
        rows = fem_ctx.sensor_rows(sensor_nodes)
        pos = out["state"][rows, 0:3]
        ctx.fem_ctx = fem_ctx
        ctx.sensors = np.asarray(sensor_nodes, np.int32)
        ctx.generation = fem_ctx.generation
        ctx.out_device = tensions.device
        ctx.out_dtype = tensions.dtype
        return torch.from_numpy(np.ascontiguousarray(pos)).to(tensions.device)

    @staticmethod
    def backward(ctx, grad_pos):
        f = ctx.fem_ctx
        if f.generation != ctx.generation:
            raise RuntimeError("the FEM context was solved or reset after this forward pass")
        g = grad_pos.detach().to("cpu", torch.float64).contiguous().numpy()
        dT, _ = f.fem_grad(ctx.sensors, g)
        grad_T = torch.from_numpy(dT).to(ctx.out_device, ctx.out_dtype)
        return grad_T, None, None, None, None, None
