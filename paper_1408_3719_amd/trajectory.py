"""Reverse mode over a run of global time steps on a fixed mesh.

A torch.autograd.Function whose forward runs n global time steps of fixed
length dt (ader_step_gts) and whose backward runs the adjoint of each step
(ader_adjoint_gts_step) in reverse order.  Only every `every`-th state is
kept on the forward pass; the states inside a segment are recomputed from its
checkpoint during the backward pass (checkpointing), so memory grows with
n / every + every states of [4][NE] doubles.  This module only schedules the
library's calls: every step and every adjoint runs in the HIP kernels.
"""
from __future__ import annotations


def gts_trajectory(solver, Q0, dt: float, n_steps: int, every: int = 10):
    """Q^n after n_steps global steps of length dt from Q0 (a device tensor
    [4][NE], float64, requires_grad allowed), differentiable with respect to
    Q0.  The solver must use a fixed mesh (mesh_velocity "eulerian"), one
    level and the Rusanov flux; dt must not exceed the smallest CFL step of
    any state on the way (the steps then all have length dt)."""
    import torch

    if n_steps < 1 or every < 1:
        raise ValueError("n_steps and every must be positive")

    def advance(Q, k0, k1):
        """State after steps k0..k1-1 from Q at step k0; all states if keep."""
        solver.upload_state(Q, k0 * dt)
        states = []
        for k in range(k0, k1):
            st = solver.step_gts((k + 1) * dt, 1)
            if abs(st["t"] - (k + 1) * dt) > 1e-12 * max(1.0, (k + 1) * dt):
                raise RuntimeError("a step was shorter than dt (dt above the CFL step)")
            states.append(solver.download_q())
        return states

    class _GTS(torch.autograd.Function):
        @staticmethod
        def forward(ctx, q0):
            q = q0.detach().to(dtype=torch.float64).contiguous()
            checkpoints = [q.clone()]
            for k0 in range(0, n_steps, every):
                k1 = min(n_steps, k0 + every)
                q = advance(q, k0, k1)[-1]
                if k1 < n_steps:
                    checkpoints.append(q.clone())
            ctx.checkpoints = checkpoints
            return q

        @staticmethod
        def backward(ctx, qbar):
            qbar = qbar.detach().to(dtype=torch.float64).contiguous()
            segments = list(range(0, n_steps, every))
            for s in reversed(range(len(segments))):
                k0 = segments[s]
                k1 = min(n_steps, k0 + every)
                start = ctx.checkpoints[s]
                states = [start] + advance(start, k0, k1)[:-1]   # state before each step
                for k in reversed(range(k1 - k0)):
                    solver.upload_state(states[k], (k0 + k) * dt)
                    qbar = solver.adjoint_gts_step(dt, qbar)
            return qbar

    return _GTS.apply(Q0)
