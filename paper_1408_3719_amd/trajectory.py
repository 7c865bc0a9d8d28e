"""Reverse mode over a run of global time steps, on a fixed mesh or on the
mesh moving with the fluid, and over macro steps of the local time stepping
on the moving mesh.

torch.autograd.Functions whose forward runs n global time steps of fixed
length dt (ader_step_gts) and whose backward runs the adjoint of each step
(ader_adjoint_gts_step, or ader_adjoint_lagrangian_step for the averages and
the node positions, at the state before that step) in reverse order.
Only every `every`-th state is kept on the forward pass; the states inside a
segment are recomputed from its checkpoint during the backward pass
(checkpointing), so memory grows with n / every + every states of [4][NE]
doubles (1.6 MB at 50k triangles; with a moving mesh also the node
positions, 0.4 MB: every = 1, keeping all states, is the cheapest choice
unless n * NE is very large).  The solver is left at some
state of the run.  lts_trajectory runs LTS macro steps recording their
schedule, and its backward replays that schedule through ader_adjoint_lts
(which keeps its own states).  This module only schedules the library's
calls: every step and every adjoint runs in the HIP kernels.
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
    if solver.cfg.mesh_velocity != "eulerian":
        raise ValueError("gts_trajectory differentiates steps on a fixed mesh; use lagrangian_trajectory")

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


def lagrangian_trajectory(solver, Q0, X0, dt: float, n_steps: int, every: int = 10):
    """(Q^n, X^n) after n_steps global steps of length dt on the mesh moving
    with the fluid, from the averages Q0 (device tensor [4][NE]) and the node
    positions X0 (device tensor (NV, 2)), differentiable with respect to both.
    The solver must use the Lagrangian mesh, one level and the Rusanov flux;
    dt must not exceed the smallest CFL step of any state on the way.
    Checkpoints hold (Q, X); a segment is recomputed from its checkpoint
    uploaded with its node positions."""
    import torch

    if n_steps < 1 or every < 1:
        raise ValueError("n_steps and every must be positive")
    if solver.cfg.mesh_velocity != "lagrangian":
        raise ValueError("lagrangian_trajectory needs the Lagrangian mesh")

    def step(k):
        st = solver.step_gts((k + 1) * dt, 1)
        if abs(st["t"] - (k + 1) * dt) > 1e-12 * max(1.0, (k + 1) * dt):
            raise RuntimeError("a step was shorter than dt (dt above the CFL step)")

    class _LAG(torch.autograd.Function):
        @staticmethod
        def forward(ctx, q0, x0):
            q = q0.detach().to(dtype=torch.float64).contiguous()
            x = x0.detach().to(dtype=torch.float64).contiguous()
            checkpoints = [(q.clone(), x.clone())]
            solver.upload_state(q, 0.0, X=x)
            for k in range(n_steps):
                step(k)
                if (k + 1) % every == 0 and k + 1 < n_steps:
                    checkpoints.append((solver.download_q(), solver.download_x()))
            ctx.checkpoints = checkpoints
            return solver.download_q(), solver.download_x()

        @staticmethod
        def backward(ctx, qbar, xbar):
            q_last, x_last = ctx.checkpoints[0]
            qbar = torch.zeros_like(q_last) if qbar is None else qbar.detach().to(torch.float64).contiguous()
            xbar = torch.zeros_like(x_last) if xbar is None else xbar.detach().to(torch.float64).contiguous()
            segments = list(range(0, n_steps, every))
            for s in reversed(range(len(segments))):
                k0 = segments[s]
                k1 = min(n_steps, k0 + every)
                states = [ctx.checkpoints[s]]            # (Q, X) before each step of the segment
                if k1 - k0 > 1:
                    solver.upload_state(states[0][0], k0 * dt, X=states[0][1])
                    for k in range(k0, k1 - 1):
                        step(k)
                        states.append((solver.download_q(), solver.download_x()))
                for k in reversed(range(k1 - k0)):
                    qbar, xbar, _, _ = solver.adjoint_lagrangian_step(dt, qbar, xbar, q=states[k][0],
                                                                      x=states[k][1])
            return qbar, xbar

    return _LAG.apply(Q0, X0)


def lts_trajectory(solver, Q0, X0, n_macro: int, t_end: float = 1e9, steps_per_element: int = 4096):
    """(Q, X) after n_macro macro steps of the solver's local time stepping
    (dyadic levels or free steps; mesh moving with the fluid, or fixed) from
    (Q0 [4][NE], X0 (NV, 2)),
    differentiable with respect to both with the schedule held fixed.  The
    forward pass records every element's steps and every macro step's tick
    length (ader_set_schedule_record); the backward pass uploads (Q0, X0),
    replays that schedule (ader_set_schedule_replay, ader_set_delta_replay)
    and runs ader_adjoint_lts, then turns the replays off.  The solver is left
    at the end state of the run."""
    import torch

    if n_macro < 1:
        raise ValueError("n_macro must be positive")

    class _LTS(torch.autograd.Function):
        @staticmethod
        def forward(ctx, q0, x0):
            q = q0.detach().to(dtype=torch.float64).contiguous()
            x = x0.detach().to(dtype=torch.float64).contiguous()
            solver.set_schedule_replay(None)
            solver.set_delta_replay(None)
            solver.upload_state(q, 0.0, X=x)
            solver.record_schedule(steps_per_element, n_macro)
            st = solver.step_lts(t_end, n_macro)
            log, deltas = solver.recorded_schedule()
            solver.record_schedule(0, 0)
            ctx.save_for_backward(q, x)
            ctx.schedule = (log, deltas, int(st["macro_steps"]))
            return solver.download_q(), solver.download_x()

        @staticmethod
        def backward(ctx, qbar, xbar):
            q0, x0 = ctx.saved_tensors
            log, deltas, n = ctx.schedule
            qbar = torch.zeros_like(q0) if qbar is None else qbar.detach().to(torch.float64).contiguous()
            xbar = torch.zeros_like(x0) if xbar is None else xbar.detach().to(torch.float64).contiguous()
            solver.set_schedule_replay(log)
            solver.set_delta_replay(deltas)
            try:
                solver.upload_state(q0, 0.0, X=x0)
                gq, gx, done = solver.adjoint_lts(n, t_end, qbar, xbar)
                if done != n:
                    raise RuntimeError("the replayed run took a different number of macro steps")
            finally:
                solver.set_schedule_replay(None)
                solver.set_delta_replay(None)
            return gq, gx

    return _LTS.apply(Q0, X0)
