"""Adjoint of one global time step on the mesh moving with the fluid through
the C ABI (ader_adjoint_lagrangian_step), dt held fixed: averages and node
positions differentiated, element by element and node by node against the
reverse-mode oracle (torch.autograd through the oracle's Lagrangian step) on
small meshes with the Rusanov and HLL fluxes (transmissive boundaries, and slip
walls with sliding and pinned nodes in the shock tube), its forward result against the oracle's step and the context's
own global step; at a larger mesh against central differences of the GPU's own
forward map and against translation invariance."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from test_oracle_adjoint import _case  # noqa: E402

from oracle.adjoint import LagrangianStep  # noqa: E402
from oracle.scheme import Config as OConfig  # noqa: E402
from oracle.scheme import GTSSolver  # noqa: E402
from workloads import explosion_case  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-10

# (the explosion at M=3 reaches a non-physical state within the step in the oracle too:
# unlimited third-order data at the jump)
CASES = [("vortex", 1), ("vortex", 2), ("vortex", 3), ("explosion", 1), ("explosion", 2), ("sod", 1), ("sod", 2)]
HLL_CASES = [("vortex", 2), ("explosion", 2), ("sod", 2)]


def _solver(mesh, Q0, M, flux="rusanov", velocity="lagrangian"):
    from paper_1408_3719_amd import Config, Solver
    return Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=M, levels=1, mesh_velocity=velocity, flux=flux))


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("name,M,flux", [c + ("rusanov",) for c in CASES] + [c + ("hll",) for c in HLL_CASES])
def test_lagrangian_adjoint_matches_reverse_mode_oracle(name, M, flux):
    mesh, Q0 = _case(name, M)
    print(f"lagrangian adjoint {name} M={M} {flux} {mesh.n_elems} triangles", flush=True)
    cfg = OConfig(M=M, levels=1, mesh_velocity="lagrangian", flux=flux)
    o = GTSSolver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
    dt = 0.5 * float(o.dtcfl.min())
    st = LagrangianStep(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    rng = np.random.default_rng(4)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    ref_q, ref_x = st.vjp(Q0, mesh.nodes, dt, qb, xb)
    ref_q1, ref_x1 = st.step(Q0, mesh.nodes, dt)
    g = _solver(mesh, Q0, M, flux=flux)
    Qa, Xa, _ = g.download()
    gq, gx, q1, x1 = (t.cpu().numpy() for t in g.adjoint_lagrangian_step(dt, qb, xb))
    gq, q1 = gq.T, q1.T
    for v in range(4):
        assert _rel(gq[:, v], ref_q[:, v]) < TOL, (v, _rel(gq[:, v], ref_q[:, v]))
    assert _rel(gx, ref_x) < TOL, _rel(gx, ref_x)
    assert _rel(q1, ref_q1) < 1e-12 and np.abs(x1 - ref_x1).max() < 1e-12 * np.ptp(mesh.nodes)
    # the simulation state is untouched; the context's own step is the one differentiated
    Qb, Xb, _ = g.download()
    assert np.array_equal(Qa, Qb) and np.array_equal(Xa, Xb)
    g.step_gts(dt, 1)
    Q1, X1, _ = g.download()
    assert _rel(Q1, q1) < 1e-12 and np.abs(X1 - x1).max() < 1e-12 * np.ptp(mesh.nodes)


def test_lagrangian_adjoint_explicit_state_and_linearity():
    """The state passed in equals the context's when they agree (bit for bit);
    the result is linear in (Qbar', Xbar'); a state reached by steps."""
    mesh, Q0 = _case("vortex", 2)
    g = _solver(mesh, Q0, 2)
    g.step_gts(10.0, 2)
    Q, X, _ = g.download()
    o = GTSSolver(X, mesh.tris, Q, OConfig(M=2, levels=1, mesh_velocity="lagrangian"), bedges=mesh.bedges)
    dt = 0.5 * float(o.dtcfl.min())
    rng = np.random.default_rng(5)
    qb = rng.standard_normal(Q.shape)
    xb = rng.standard_normal(X.shape)
    a = [t.cpu().numpy() for t in g.adjoint_lagrangian_step(dt, qb, xb)]
    b = [t.cpu().numpy() for t in g.adjoint_lagrangian_step(dt, qb, xb, q=Q, x=X)]
    for u, w in zip(a, b):
        assert np.array_equal(u, w)
    c = [t.cpu().numpy() for t in g.adjoint_lagrangian_step(dt, 2.0 * qb, -3.0 * xb)]
    d = [t.cpu().numpy() for t in g.adjoint_lagrangian_step(dt, 0.0 * qb, xb)]
    e = [t.cpu().numpy() for t in g.adjoint_lagrangian_step(dt, qb, 0.0 * xb)]
    for k in range(2):
        lin = 2.0 * e[k] - 3.0 * d[k]
        assert np.abs(c[k] - lin).max() <= 1e-12 * np.abs(lin).max()
        assert np.abs(a[k] - (d[k] + e[k])).max() <= 1e-12 * np.abs(a[k]).max()
    # the stencils are fixed on the initial mesh (the context's), not rebuilt on X
    o0 = GTSSolver(mesh.nodes, mesh.tris, Q0, OConfig(M=2, levels=1, mesh_velocity="lagrangian"),
                   bedges=mesh.bedges)
    st = LagrangianStep(X, mesh.tris, OConfig(M=2, levels=1, mesh_velocity="lagrangian"), bedges=mesh.bedges,
                        topo=o0.topo)
    rq, rx = st.vjp(Q, X, dt, qb, xb)
    assert _rel(a[0].T, rq) < TOL and _rel(a[1], rx) < TOL


def test_lagrangian_adjoint_central_differences_and_translation():
    """20k-triangle explosion, M=2: <Qbar, v> + <Xbar, y> against central
    differences of the forward map the same entry point returns (h = 1e-7
    relative), in the averages, the positions and both; the position adjoints
    sum to the sum of Xbar' (translation invariance)."""
    mesh, Q0 = explosion_case(20000, seed=9)
    rng = np.random.default_rng(6)
    Q0 = Q0 * (1.0 + 1e-3 * rng.standard_normal(Q0.shape))
    print(f"lagrangian adjoint FD: {mesh.n_elems} triangles", flush=True)
    g = _solver(mesh, Q0, 2)
    o = GTSSolver(mesh.nodes, mesh.tris, Q0, OConfig(M=2, levels=1, mesh_velocity="lagrangian"),
                  bedges=mesh.bedges)
    dt = 0.5 * float(o.dtcfl.min())
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    gq, gx, _, _ = (t.cpu().numpy() for t in g.adjoint_lagrangian_step(dt, qb, xb))
    gq = gq.T
    assert np.abs(gx.sum(axis=0) - xb.sum(axis=0)).max() <= 1e-11 * np.abs(gx).sum(axis=0).max()

    def F(Q, X):
        _, _, q1, x1 = g.adjoint_lagrangian_step(dt, qb, xb, q=Q, x=X)
        return q1.cpu().numpy().T, x1.cpu().numpy()

    h = 1e-7
    span = np.ptp(mesh.nodes)
    for k, (wq, wx) in enumerate(((1, 1), (1, 0), (0, 1))):
        v = wq * rng.standard_normal(Q0.shape) * np.abs(Q0).max(axis=0)
        y = wx * rng.standard_normal(mesh.nodes.shape) * 1e-3 * span
        Qp, Xp = F(Q0 + h * v, mesh.nodes + h * y)
        Qm, Xm = F(Q0 - h * v, mesh.nodes - h * y)
        fd = (((Qp - Qm) * qb).sum() + ((Xp - Xm) * xb).sum()) / (2 * h)
        ad = (gq * v).sum() + (gx * y).sum()
        scale = np.abs(gq * v).sum() + np.abs(gx * y).sum()
        print(f"direction {k}: fd {fd:.12e} adjoint {ad:.12e} rel {abs(fd - ad) / scale:.2e}", flush=True)
        assert abs(fd - ad) <= 1e-6 * scale, (k, fd, ad)


def test_lagrangian_adjoint_rejects_unsupported_modes():
    from paper_1408_3719_amd import AderError
    mesh, Q0 = _case("vortex", 2)
    qb = np.zeros(Q0.shape)
    xb = np.zeros(mesh.nodes.shape)
    for kw in ({"velocity": "eulerian"}, {"flux": "osher"}):
        g = _solver(mesh, Q0, 2, **kw)
        with pytest.raises(AderError):
            g.adjoint_lagrangian_step(1e-4, qb, xb)
    g = _solver(*_case("vortex", 2), 2)
    with pytest.raises(AderError, match="dt"):
        g.adjoint_lagrangian_step(-1.0, qb, xb)


def test_upload_state_with_node_positions_restores_a_moved_mesh():
    """A state of a Lagrangian run (averages and moved nodes) uploaded into a
    fresh context continues exactly as the original run (bit for bit);
    positions that invert the elements are refused."""
    from paper_1408_3719_amd import AderError
    mesh, Q0 = _case("vortex", 2)
    g = _solver(mesh, Q0, 2)
    t3 = g.step_gts(10.0, 3)["t"]
    Q3, X3 = g.download_q(), g.download_x()
    g.step_gts(10.0, 2)
    Q5, X5, _ = g.download()
    h = _solver(mesh, Q0, 2)
    h.upload_state(Q3, t3, X=X3)
    assert np.array_equal(h.download_x().cpu().numpy(), X3.cpu().numpy())
    h.step_gts(10.0, 2)
    Qh, Xh, _ = h.download()
    assert np.array_equal(Qh, Q5) and np.array_equal(Xh, X5)
    with pytest.raises(AderError, match="inverted"):
        h.upload_state(Q3, t3, X=X3.cpu().numpy() * np.array([-1.0, 1.0]))     # mirrored: every element inverted


@pytest.mark.parametrize("every", [1, 2])
def test_lagrangian_trajectory_gradient_matches_oracle(every):
    """Gradient of a weighted sum of (Q^3, X^3) with respect to (Q^0, X^0)
    through three Lagrangian global steps (torch.autograd.Function over the
    library's steps and adjoints, checkpoints every `every` steps) against
    autograd through three oracle steps."""
    import torch

    from paper_1408_3719_amd.trajectory import lagrangian_trajectory
    mesh, Q0 = _case("vortex", 2)
    cfg = OConfig(M=2, levels=1, mesh_velocity="lagrangian")
    o = GTSSolver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
    dt = 0.4 * float(o.dtcfl.min())
    st = LagrangianStep(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    rng = np.random.default_rng(8)
    Wq = rng.standard_normal(Q0.shape)
    Wx = rng.standard_normal(mesh.nodes.shape)
    q = torch.tensor(Q0, dtype=torch.float64, requires_grad=True)
    x = torch.tensor(mesh.nodes, dtype=torch.float64, requires_grad=True)
    qk, xk = q, x
    for _ in range(3):
        qk, xk = st(qk, xk, dt)
    ((qk * torch.tensor(Wq)).sum() + (xk * torch.tensor(Wx)).sum()).backward()
    ref = (qk.detach().numpy(), xk.detach().numpy(), q.grad.numpy(), x.grad.numpy())

    g = _solver(mesh, Q0, 2)
    q0 = torch.tensor(Q0.T.copy(), dtype=torch.float64, device="cuda", requires_grad=True)
    x0 = torch.tensor(mesh.nodes, dtype=torch.float64, device="cuda", requires_grad=True)
    q3, x3 = lagrangian_trajectory(g, q0, x0, dt, 3, every=every)
    ((q3 * torch.tensor(Wq.T.copy(), device="cuda")).sum() + (x3 * torch.tensor(Wx, device="cuda")).sum()).backward()
    got = (q3.detach().cpu().numpy().T, x3.detach().cpu().numpy(), q0.grad.cpu().numpy().T, x0.grad.cpu().numpy())
    assert _rel(got[0], ref[0]) < 1e-12 and _rel(got[1], ref[1]) < 1e-12
    for v in range(4):
        assert _rel(got[2][:, v], ref[2][:, v]) < TOL, (v, _rel(got[2][:, v], ref[2][:, v]))
    assert _rel(got[3], ref[3]) < TOL, _rel(got[3], ref[3])


def _fixed_dt(s, n_steps):
    """0.8 x the smallest of n_steps global CFL steps from the uploaded state
    (the Lagrangian mesh compresses, so the CFL step shrinks along the run; a
    shorter fixed step evolves less and stays below it)."""
    t = [0.0] + [s.step_gts(1e9, 1)["t"] for _ in range(n_steps)]
    return 0.8 * float(np.diff(t).min())


def _inner_energy(mesh):
    """J(Q, X) = sum over the elements whose initial centroid lies in r < 0.3
    of |T(X)| (rho E): the total energy they carry (torch, on the device)."""
    import torch
    c = mesh.nodes[mesh.tris].mean(axis=1)
    inner = torch.tensor(np.nonzero(np.hypot(c[:, 0], c[:, 1]) < 0.3)[0], device="cuda")
    tris = torch.tensor(mesh.tris, dtype=torch.long, device="cuda")[inner]

    def J(q, x):
        p = x[tris]
        A = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                   - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
        return (A * q[3][inner]).sum()
    return J


def test_lagrangian_explosion_100_steps_gradient_against_central_differences():
    """The moving-mesh adjoint workload: 50k-triangle explosion, M=2, 100
    Lagrangian global steps with checkpoints every 10 steps; J = energy carried
    by the elements that start inside r < 0.3, at the final time (their moved
    areas included); dJ/d(initial density) on 32 seeded directions and
    dJ/d(initial node positions) on 8, against central differences (h = 1e-6
    relative) of the library's own forward run; dt fixed at 0.8 x the smallest
    CFL step of 100 free-running global steps."""
    import torch

    from paper_1408_3719_amd.trajectory import lagrangian_trajectory
    mesh, Q0 = explosion_case(50_000, seed=7)
    NE = mesh.n_elems
    rng = np.random.default_rng(12)
    Q0 = Q0 * (1.0 + 1e-3 * rng.standard_normal(Q0.shape))
    J = _inner_energy(mesh)
    s = _solver(mesh, Q0, 2)
    dt = _fixed_dt(s, 100)
    q0 = torch.tensor(Q0.T.copy(), device="cuda", requires_grad=True)
    x0 = torch.tensor(mesh.nodes, device="cuda", requires_grad=True)
    J(*lagrangian_trajectory(s, q0, x0, dt, 100, every=10)).backward()
    gq = q0.grad[0].cpu().numpy()
    gx = x0.grad.cpu().numpy()
    assert np.isfinite(gq).all() and np.isfinite(gx).all()

    def run(Q, X):
        s.upload_state(Q, 0.0, X=X)
        for k in range(100):
            s.step_gts((k + 1) * dt, 1)
        return float(J(s.download_q(), s.download_x()))

    h = 1e-6
    worst = 0.0
    for d in range(32):
        v = rng.standard_normal(NE) * Q0[:, 0]
        Qp, Qm = Q0.copy(), Q0.copy()
        Qp[:, 0] += h * v
        Qm[:, 0] -= h * v
        fd = (run(Qp, mesh.nodes) - run(Qm, mesh.nodes)) / (2 * h)
        worst = max(worst, abs(fd - float((gq * v).sum())) / np.abs(gq * v).sum())
    span = np.ptp(mesh.nodes)
    worst_x = 0.0
    for d in range(8):
        y = rng.standard_normal(mesh.nodes.shape) * 1e-3 * span
        fd = (run(Q0, mesh.nodes + h * y) - run(Q0, mesh.nodes - h * y)) / (2 * h)
        worst_x = max(worst_x, abs(fd - float((gx * y).sum())) / np.abs(gx * y).sum())
    print(f"density: 32 directions, worst {worst:.2e}; positions: 8 directions, worst {worst_x:.2e}", flush=True)
    assert worst < 1e-5 and worst_x < 1e-5
