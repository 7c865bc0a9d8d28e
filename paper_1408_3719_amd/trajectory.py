"""Reverse mode over a run of global time steps on a fixed mesh.

A torch.autograd.Function whose forward runs n global time steps of fixed
length dt (ader_step_gts) and whose backward runs the adjoint of each step
(ader_adjoint_gts_step, at the state before that step) in reverse order.
Only every `every`-th state is kept on the forward pass; the states inside a
segment are recomputed from its checkpoint during the backward pass
(checkpointing), so memory grows with n / every + every states of [4][NE]
doubles (1.6 MB at 50k triangles: every = 1, keeping all states, is the
cheapest choice unless n * NE is very large).  The solver is left at some
state of the run.  This module only schedules the library's calls: every
step and every adjoint runs in the HIP kernels.
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

    def step(k):
        st = solver.step_gts((k + 1) * dt, 1)
        if abs(st["t"] - (k + 1) * dt) > 1e-12 * max(1.0, (k + 1) * dt):
            raise RuntimeError("a step was shorter than dt (dt above the CFL step)")

    class _GTS(torch.autograd.Function):
        @staticmethod
        def forward(ctx, q0):
            q = q0.detach().to(dtype=torch.float64).contiguous()
            checkpoints = [q.clone()]
            solver.upload_state(q, 0.0)
            for k in range(n_steps):
                step(k)
                if (k + 1) % every == 0 and k + 1 < n_steps:
                    checkpoints.append(solver.download_q())
            ctx.checkpoints = checkpoints
            return solver.download_q()

        @staticmethod
        def backward(ctx, qbar):
            qbar = qbar.detach().to(dtype=torch.float64).contiguous()
            segments = list(range(0, n_steps, every))
            for s in reversed(range(len(segments))):
                k0 = segments[s]
                k1 = min(n_steps, k0 + every)
                states = [ctx.checkpoints[s]]            # the state before each step of the segment
                if k1 - k0 > 1:
                    solver.upload_state(states[0], k0 * dt)
                    for k in range(k0, k1 - 1):
                        step(k)
                        states.append(solver.download_q())
                for k in reversed(range(k1 - k0)):
                    qbar = solver.adjoint_gts_step(dt, qbar, q=states[k])
            return qbar

    return _GTS.apply(Q0)
