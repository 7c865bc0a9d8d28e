"""Pins of the reverse-mode oracle of the local time stepping scheme
(oracle/adjoint.py: LagrangianLTS): dyadic macro steps on a mesh moving with
the fluid (and on a fixed mesh), with the schedule held fixed (tick length and every element's
steps).  Its forward map must equal the NumPy oracle's LTS solver, one level
must reduce to global steps, its vector-Jacobian product must match central
differences of the NumPy solver replaying the same schedule, and a translation
of every node must leave the averages unchanged."""
import numpy as np
import pytest

from oracle.adjoint import LagrangianLTS, LagrangianStep, lts_schedule
from oracle.scheme import Config, MACRO_TICKS, Solver
from workloads import explosion_case, sod_case, vortex_case


def _case(name):
    rng = np.random.default_rng(3)
    if name == "vortex":
        mesh, Q0 = vortex_case(300, seed=5)
    elif name == "sod":
        mesh, Q0 = sod_case(300, seed=11)
    else:
        mesh, Q0 = explosion_case(1500, seed=7)
    # break the exact ties of the piecewise-constant data (max and |.| kinks)
    return mesh, Q0 * (1.0 + 1e-3 * rng.standard_normal(Q0.shape))


def _setup(name, levels=3, n_macro=2, flux="rusanov", M=2, mode="lagrangian"):
    mesh, Q0 = _case(name)
    cfg = Config(M=M, levels=levels, mesh_velocity=mode, flux=flux)
    o = Solver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
    sched = lts_schedule(o, 10.0, n_macro)
    lt = LagrangianLTS(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    return mesh, Q0, cfg, o, sched, lt


def _replay(mesh, cfg, topo, sched, Q, X, t_end=10.0):
    """The NumPy solver from (Q, X) taking the recorded steps and tick lengths."""
    steps = [sum((list(s[i]) for _, s in sched), []) for i in range(len(Q))]
    s = Solver(X, mesh.tris, Q, cfg, bedges=mesh.bedges, topo=topo)
    s.step_hook = lambda i, k, p: steps[i][k]
    s.delta_hook = lambda m: sched[m][0]
    for _ in sched:
        s.macro_step(t_end)
    return s.st.Q, s.st.X


@pytest.mark.parametrize("name,M", [("vortex", 1), ("vortex", 2), ("vortex", 3), ("sod", 2), ("explosion", 2)])
def test_lts_forward_equals_numpy_solver(name, M):
    mesh, Q0, cfg, o, sched, lt = _setup(name, M=M)
    assert o.st.cycles > 2 * 4 - 1 and o.st.updates > 2 * len(Q0)   # several levels are in use
    Q, X = lt.run(Q0, mesh.nodes, sched)
    assert np.abs(Q - o.st.Q).max() <= 1e-14 * np.abs(o.st.Q).max()
    assert np.abs(X - o.st.X).max() <= 1e-14 * np.abs(o.st.X).max()


@pytest.mark.parametrize("name", ["vortex", "explosion"])
def test_lts_fixed_mesh_forward_and_central_differences(name):
    """The same macro step on a fixed mesh (V = 0 in the mesh ODE, nodes at
    rest, their ticks still advancing): the forward equals the NumPy LTS
    solver in Eulerian mode, and the product matches central differences of
    the NumPy solver replaying the schedule (averages and node positions)."""
    mesh, Q0, cfg, o, sched, lt = _setup(name, mode="eulerian")
    Q, X = lt.run(Q0, mesh.nodes, sched)
    assert np.abs(Q - o.st.Q).max() <= 1e-14 * np.abs(o.st.Q).max()
    assert np.array_equal(X, mesh.nodes) and np.array_equal(o.st.X, mesh.nodes)
    rng = np.random.default_rng(4)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    gq, gx = lt.vjp(Q0, mesh.nodes, sched, qb, xb)
    h = 1e-8
    v = rng.standard_normal(Q0.shape) * np.abs(Q0).max(axis=0)
    y = rng.standard_normal(mesh.nodes.shape) * np.ptp(mesh.nodes) * 1e-1
    Qp, Xp = _replay(mesh, cfg, o.topo, sched, Q0 + h * v, mesh.nodes + h * y)
    Qm, Xm = _replay(mesh, cfg, o.topo, sched, Q0 - h * v, mesh.nodes - h * y)
    fd = (((Qp - Qm) * qb).sum() + ((Xp - Xm) * xb).sum()) / (2 * h)
    ad = (gq * v).sum() + (gx * y).sum()
    assert abs(fd - ad) <= 1e-6 * (np.abs(gq * v).sum() + np.abs(gx * y).sum()), (fd, ad)


def test_lts_free_steps_forward_and_central_differences():
    """Free local steps (levels = 0: one macro step of 2^30 ticks to the
    target time, every element at its own CFL step): the forward equals the
    NumPy solver, and the product matches central differences of the NumPy
    solver replaying the schedule."""
    mesh, Q0 = _case("vortex")
    cfg = Config(M=2, levels=0, mesh_velocity="lagrangian")
    o = Solver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
    sched = lts_schedule(o, 0.05, 1)
    assert o.st.cycles > 4 and o.st.updates > len(Q0)       # elements at different steps
    lt = LagrangianLTS(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    Q, X = lt.run(Q0, mesh.nodes, sched)
    assert np.abs(Q - o.st.Q).max() <= 1e-14 * np.abs(o.st.Q).max()
    assert np.abs(X - o.st.X).max() <= 1e-14 * np.abs(o.st.X).max()
    rng = np.random.default_rng(5)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    gq, gx = lt.vjp(Q0, mesh.nodes, sched, qb, xb)
    h = 1e-8
    v = rng.standard_normal(Q0.shape) * np.abs(Q0).max(axis=0)
    y = rng.standard_normal(mesh.nodes.shape) * np.ptp(mesh.nodes) * 1e-1
    Qp, Xp = _replay(mesh, cfg, o.topo, sched, Q0 + h * v, mesh.nodes + h * y, t_end=0.05)
    Qm, Xm = _replay(mesh, cfg, o.topo, sched, Q0 - h * v, mesh.nodes - h * y, t_end=0.05)
    fd = (((Qp - Qm) * qb).sum() + ((Xp - Xm) * xb).sum()) / (2 * h)
    ad = (gq * v).sum() + (gx * y).sum()
    assert abs(fd - ad) <= 1e-6 * (np.abs(gq * v).sum() + np.abs(gx * y).sum()), (fd, ad)


def test_lts_one_level_is_the_global_step():
    """With one level every macro step is one cycle in which every element is
    updated over N ticks: the global Lagrangian step of length N delta."""
    mesh, Q0, cfg, o, sched, lt = _setup("vortex", levels=1)
    Q, X = lt.run(Q0, mesh.nodes, sched)
    g = LagrangianStep(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    Qg, Xg = Q0, mesh.nodes
    for delta, _ in sched:
        Qg, Xg = g.step(Qg, Xg, MACRO_TICKS * delta)
    assert np.abs(Q - Qg).max() <= 1e-14 * np.abs(Qg).max()
    assert np.abs(X - Xg).max() <= 1e-14 * np.abs(Xg).max()


@pytest.mark.parametrize("name", ["vortex", "explosion"])
def test_lts_vjp_matches_central_differences(name):
    """<(Qbar, Xbar), (F(Q+hv, X+hy) - F(Q-hv, X-hy)) / 2h> of the NumPy LTS
    solver replaying the schedule against the vector-Jacobian product, with
    directions in the averages and the node positions together and alone.
    (Not the shock tube: on its slip walls the mirrored state has the inner
    state's signal speed, an exact tie in the Rusanov maximum, where central
    differences see the mean of the two one-sided derivatives.)"""
    mesh, Q0, cfg, o, sched, lt = _setup(name)
    rng = np.random.default_rng(1)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    gq, gx = lt.vjp(Q0, mesh.nodes, sched, qb, xb)
    h = 1e-8
    hx = h * np.ptp(mesh.nodes) * 1e-1
    for k, (wq, wx) in enumerate(((1, 1), (1, 0), (0, 1))):
        v = wq * rng.standard_normal(Q0.shape) * np.abs(Q0).max(axis=0)
        y = wx * rng.standard_normal(mesh.nodes.shape) * hx / h
        Qp, Xp = _replay(mesh, cfg, o.topo, sched, Q0 + h * v, mesh.nodes + h * y)
        Qm, Xm = _replay(mesh, cfg, o.topo, sched, Q0 - h * v, mesh.nodes - h * y)
        fd = (((Qp - Qm) * qb).sum() + ((Xp - Xm) * xb).sum()) / (2 * h)
        ad = (gq * v).sum() + (gx * y).sum()
        scale = np.abs(gq * v).sum() + np.abs(gx * y).sum()
        assert abs(fd - ad) <= 1e-6 * scale, (k, fd, ad)


def test_lts_adjoint_of_a_translation():
    """Moving every node by one vector moves every node after the macro steps
    by it and leaves the averages unchanged: the node-position adjoints sum to
    the sum of Xbar."""
    mesh, Q0, cfg, o, sched, lt = _setup("explosion")
    rng = np.random.default_rng(2)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    _, gx = lt.vjp(Q0, mesh.nodes, sched, qb, xb)
    scale = np.abs(gx).sum(axis=0)
    assert np.abs(gx.sum(axis=0) - xb.sum(axis=0)).max() <= 1e-12 * scale.max()
    assert np.abs(gx - xb).max() > 1e-3 * np.abs(xb).max()
