"""Gradient through macro steps of the local time stepping on the mesh moving
with the fluid, through the C ABI (ader_adjoint_lts), the schedule held fixed:
averages and node positions of the uploaded state, element by element and node
by node against the reverse-mode oracle (torch.autograd through the oracle's
LTS macro steps replaying the same tick lengths and steps) on small meshes with
three levels (vortex M = 1, 2, 3, explosion, shock tube with slip walls; Rusanov, and HLL on the
explosion; also on a fixed mesh); the context's end state
against the oracle's forward run; macro steps with their cycle states kept and
macro steps replayed from their start against each other; with one level
against the adjoint of the global Lagrangian step (ader_adjoint_lagrangian_step)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from test_oracle_adjoint_lts import _case  # noqa: E402

from oracle.adjoint import LagrangianLTS, lts_schedule  # noqa: E402
from oracle.scheme import Config as OConfig  # noqa: E402
from oracle.scheme import Solver as OSolver  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _gpu(mesh, Q0, levels, flux, M=2, mode="lagrangian"):
    from paper_1408_3719_amd import Config, Solver
    return Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0,
                  Config(M=M, levels=levels, mesh_velocity=mode, flux=flux))


@pytest.mark.parametrize("name,M,flux,mode", [("vortex", 2, "rusanov", "lagrangian"),
                                              ("explosion", 2, "rusanov", "lagrangian"),
                                              ("explosion", 2, "hll", "lagrangian"),
                                              ("vortex", 1, "rusanov", "lagrangian"),
                                              ("vortex", 3, "rusanov", "lagrangian"),
                                              ("sod", 2, "rusanov", "lagrangian"),
                                              ("vortex", 2, "rusanov", "eulerian"),
                                              ("explosion", 2, "hll", "eulerian")])
def test_lts_adjoint_matches_reverse_mode_oracle(name, M, flux, mode):
    mesh, Q0 = _case(name)
    print(f"lts adjoint {name} M={M} {flux} {mode} {mesh.n_elems} triangles, 3 levels, 2 macro steps", flush=True)
    cfg = OConfig(M=M, levels=3, mesh_velocity=mode, flux=flux)
    o = OSolver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
    sched = lts_schedule(o, 10.0, 2)
    lt = LagrangianLTS(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    rng = np.random.default_rng(6)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    ref_q, ref_x = lt.vjp(Q0, mesh.nodes, sched, qb, xb)
    g = _gpu(mesh, Q0, 3, flux, M, mode)
    g.set_schedule_replay(o.step_log)
    gq, gx, done = g.adjoint_lts(2, 10.0, qb, xb)
    assert done == 2
    gq, gx = gq.cpu().numpy().T, gx.cpu().numpy()
    for v in range(4):
        assert _rel(gq[:, v], ref_q[:, v]) < TOL, (v, _rel(gq[:, v], ref_q[:, v]))
    assert _rel(gx, ref_x) < TOL, _rel(gx, ref_x)
    # the context ends where the forward run ends
    Q, X, _ = g.download()
    assert _rel(Q, o.st.Q) < 1e-12 and np.abs(X - o.st.X).max() < 1e-12 * np.ptp(mesh.nodes)
    assert g.stats()["element_updates"] == o.st.updates


def test_lts_adjoint_replayed_and_kept_macro_steps_agree():
    """Macro steps whose cycle states are kept and macro steps replayed from
    their saved start give the same gradient (and the same end state)."""
    mesh, Q0 = _case("explosion")
    rng = np.random.default_rng(8)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    out = []
    for keep in (-1, 0, 1):
        g = _gpu(mesh, Q0, 3, "rusanov")
        gq, gx, done = g.adjoint_lts(3, 10.0, qb, xb, keep=keep)
        assert done == 3
        Q, X, _ = g.download()
        out.append((gq.cpu().numpy(), gx.cpu().numpy(), Q, X))
    for o in out[1:]:
        assert _rel(o[0], out[0][0]) < 1e-13 and _rel(o[1], out[0][1]) < 1e-13
        assert np.array_equal(o[2], out[0][2]) and np.array_equal(o[3], out[0][3])


def test_lts_adjoint_one_level_is_the_global_step_adjoint():
    """One level: a macro step is one global step of length N delta, whose
    reconstruction is the pre-processing one; the two adjoints agree."""
    mesh, Q0 = _case("explosion")
    rng = np.random.default_rng(7)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    g = _gpu(mesh, Q0, 1, "rusanov")
    gq, gx, done = g.adjoint_lts(1, 10.0, qb, xb)
    assert done == 1
    T1 = g.stats()["t"]
    h = _gpu(mesh, Q0, 1, "rusanov")
    hq, hx, _, _ = h.adjoint_lagrangian_step(T1, qb, xb)
    assert _rel(gq.cpu().numpy(), hq.cpu().numpy()) < 1e-11
    assert _rel(gx.cpu().numpy(), hx.cpu().numpy()) < 1e-11


def test_lts_adjoint_errors():
    from paper_1408_3719_amd import AderError
    mesh, Q0 = _case("vortex")
    g = _gpu(mesh, Q0, 3, "rusanov")
    qb = np.zeros(Q0.shape)
    xb = np.zeros(mesh.nodes.shape)
    g.step_lts(10.0, 1)
    with pytest.raises(AderError, match="uploaded state"):
        g.adjoint_lts(1, 10.0, qb, xb)
    with pytest.raises(AderError, match="Rusanov and HLL"):
        _gpu(mesh, Q0, 3, "osher").adjoint_lts(1, 10.0, qb, xb)



def test_lts_gradient_of_the_adjoint_workload_against_central_differences():
    """The adjoint workload with LTS: explosion recipe at 50k triangles (data
    times 1 + 1e-3 seeded noise, so that density moves pressure and
    velocity), M=2, 3 levels, 100 macro steps from t = 0, J = energy carried
    at the end by the elements that start inside r < 0.3; the gradient with
    respect to the initial densities on 32 seeded directions and the initial
    node positions on 8, against central differences (h = 1e-6 relative) of
    the library's own forward run, and again with h = 1e-7 on the four
    directions that deviate most (the deviation is the differences'
    truncation error, falling as h^2); the perturbed runs replay the recorded
    steps and tick lengths (the schedule held fixed)."""
    from test_gpu_adjoint_lagrangian import _inner_energy
    from workloads import explosion_case
    mesh, Q0 = explosion_case(50_000, seed=7)
    rng = np.random.default_rng(12)
    Q0 = Q0 * (1.0 + 1e-3 * rng.standard_normal(Q0.shape))
    n_macro = 100
    J = _inner_energy(mesh)
    g = _gpu(mesh, Q0, 3, "rusanov")
    g.record_schedule(4096, n_macro)
    g.step_lts(1e9, n_macro)
    log, deltas = g.recorded_schedule()
    assert len(deltas) == n_macro
    q = g.download_q().clone().requires_grad_(True)
    x = g.download_x().clone().requires_grad_(True)
    J(q, x).backward()
    g.record_schedule(0, 0)
    g.set_schedule_replay(log)
    g.set_delta_replay(deltas)
    g.upload_state(Q0, 0.0)
    gq, gx, done = g.adjoint_lts(n_macro, 1e9, q.grad, x.grad)
    assert done == n_macro
    grad_rho, gx = gq[0].cpu().numpy(), gx.cpu().numpy()

    def run(Q, X):
        g.set_schedule_replay(log)
        g.upload_state(Q, 0.0, X=X)
        g.step_lts(1e9, n_macro)
        assert g.stats()["macro_steps"] == n_macro
        return float(J(g.download_q(), g.download_x()))

    def dev(v, h):
        Qp, Qm = Q0.copy(), Q0.copy()
        Qp[:, 0] += h * v
        Qm[:, 0] -= h * v
        fd = (run(Qp, mesh.nodes) - run(Qm, mesh.nodes)) / (2 * h)
        return abs(fd - float((grad_rho * v).sum())) / float(np.abs(grad_rho * v).sum())

    h = 1e-6
    dirs = [rng.standard_normal(mesh.n_elems) * Q0[:, 0] for _ in range(32)]
    devs = [dev(v, h) for v in dirs]
    worst = max(devs)
    # the deviation is the differences' truncation error: it falls as h^2
    # (measured: ~1e-4 at h = 1e-5, ~1e-6 at 1e-6, ~1e-7 at 1e-7, rounding)
    finer = [dev(dirs[k], 1e-7) for k in np.argsort(devs)[-4:]]
    span = np.ptp(mesh.nodes)
    worst_x = 0.0
    for k in range(8):
        y = rng.standard_normal(mesh.nodes.shape) * 1e-3 * span
        fd = (run(Q0, mesh.nodes + h * y) - run(Q0, mesh.nodes - h * y)) / (2 * h)
        worst_x = max(worst_x, abs(fd - float((gx * y).sum())) / float(np.abs(gx * y).sum()))
    print(f"LTS adjoint workload: density 32 directions, worst {worst:.2e} (h = 1e-7 on the worst four: "
          f"{max(finer):.2e}); positions 8 directions, worst {worst_x:.2e}", flush=True)
    assert worst < 3e-5 and max(finer) < 1e-6 and worst_x < 1e-5


def test_lts_trajectory_autograd_and_linearity():
    """paper_1408_3719_amd.trajectory.lts_trajectory: its forward is the
    library's LTS run, its gradient (torch.autograd through the recorded and
    replayed schedule) equals ader_adjoint_lts with that schedule, and the
    adjoint is linear in (Qbar, Xbar): adj(a w1 + b w2) = a adj(w1) + b adj(w2)."""
    import torch

    from paper_1408_3719_amd.trajectory import lts_trajectory
    mesh, Q0 = _case("explosion")
    g = _gpu(mesh, Q0, 3, "rusanov")
    rng = np.random.default_rng(10)
    w1 = torch.tensor(rng.standard_normal((4, mesh.n_elems)), device="cuda")
    y1 = torch.tensor(rng.standard_normal(mesh.nodes.shape), device="cuda")
    w2 = torch.tensor(rng.standard_normal((4, mesh.n_elems)), device="cuda")
    y2 = torch.tensor(rng.standard_normal(mesh.nodes.shape), device="cuda")
    q0 = torch.tensor(Q0.T.copy(), device="cuda", requires_grad=True)
    x0 = torch.tensor(mesh.nodes, device="cuda", requires_grad=True)
    qn, xn = lts_trajectory(g, q0, x0, 2, t_end=10.0)
    ((w1 * qn).sum() + (y1 * xn).sum()).backward()
    h = _gpu(mesh, Q0, 3, "rusanov")
    h.step_lts(10.0, 2)
    Q, X, _ = h.download()
    assert np.array_equal(qn.detach().cpu().numpy().T, Q) and np.array_equal(xn.detach().cpu().numpy(), X)
    h.record_schedule(64, 4)
    h.upload_state(Q0, 0.0)
    h.step_lts(10.0, 2)
    log, deltas = h.recorded_schedule()
    h.record_schedule(0, 0)

    def adj(qb, xb):
        h.set_schedule_replay(log)
        h.set_delta_replay(deltas)
        h.upload_state(Q0, 0.0)
        gq, gx, done = h.adjoint_lts(2, 10.0, qb, xb)
        assert done == 2
        return gq.cpu().numpy(), gx.cpu().numpy()

    gq1, gx1 = adj(w1, y1)
    assert _rel(q0.grad.cpu().numpy(), gq1) < 1e-13 and _rel(x0.grad.cpu().numpy(), gx1) < 1e-13
    gq2, gx2 = adj(w2, y2)
    gq3, gx3 = adj(2.0 * w1 - 0.5 * w2, 2.0 * y1 - 0.5 * y2)
    assert _rel(gq3, 2.0 * gq1 - 0.5 * gq2) < 1e-12 and _rel(gx3, 2.0 * gx1 - 0.5 * gx2) < 1e-12


def test_lts_adjoint_stops_at_the_target_time():
    """With t_end reached after fewer macro steps than asked, the gradient is
    the one through the macro steps taken (the oracle's over the same run)."""
    mesh, Q0 = _case("vortex")
    cfg = OConfig(M=2, levels=3, mesh_velocity="lagrangian")
    o = OSolver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
    sched = lts_schedule(o, 10.0, 1)
    t1 = o.st.T
    o2 = OSolver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges, topo=o.topo)
    sched = lts_schedule(o2, 1.5 * t1, 2)       # the second macro step is cut at 1.5 t1
    assert abs(o2.st.T - 1.5 * t1) <= 1e-12 * t1
    lt = LagrangianLTS(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    rng = np.random.default_rng(11)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    ref_q, ref_x = lt.vjp(Q0, mesh.nodes, sched, qb, xb)
    g = _gpu(mesh, Q0, 3, "rusanov")
    g.set_schedule_replay(o2.step_log)
    gq, gx, done = g.adjoint_lts(5, 1.5 * t1, qb, xb)
    assert done == 2
    assert abs(g.stats()["t"] - 1.5 * t1) <= 1e-12 * t1
    gq, gx = gq.cpu().numpy().T, gx.cpu().numpy()
    assert _rel(gq, ref_q) < TOL and _rel(gx, ref_x) < TOL


@pytest.mark.parametrize("mode", ["lagrangian", "eulerian"])
def test_lts_adjoint_with_free_steps(mode):
    """Free local steps (levels = 0: one macro step to the target time, each
    element at its own CFL step, reading of the paper's LTS) against the
    reverse-mode oracle with the oracle's schedule replayed."""
    mesh, Q0 = _case("vortex")
    cfg = OConfig(M=2, levels=0, mesh_velocity=mode)
    o = OSolver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
    sched = lts_schedule(o, 0.05, 1)
    lt = LagrangianLTS(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    rng = np.random.default_rng(13)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    ref_q, ref_x = lt.vjp(Q0, mesh.nodes, sched, qb, xb)
    g = _gpu(mesh, Q0, 0, "rusanov", mode=mode)
    g.set_schedule_replay(o.step_log)
    gq, gx, done = g.adjoint_lts(1, 0.05, qb, xb)
    assert done == 1 and abs(g.stats()["t"] - 0.05) <= 1e-14
    gq, gx = gq.cpu().numpy().T, gx.cpu().numpy()
    assert _rel(gq, ref_q) < TOL and _rel(gx, ref_x) < TOL
    Q, X, _ = g.download()
    assert _rel(Q, o.st.Q) < 1e-12 and np.abs(X - o.st.X).max() < 1e-12 * np.ptp(mesh.nodes)
