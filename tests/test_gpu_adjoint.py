"""Adjoint of one global time step on a fixed mesh through the C ABI
(ader_adjoint_gts_step), dt held fixed: element by element against the
reverse-mode oracle (torch.autograd through the oracle's step) on small
meshes; at the benchmark's mesh size against central differences of the GPU's
own forward step and against the conservation identity of the adjoint."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from test_oracle_adjoint import CASES, HLL_CASES, _case  # noqa: E402

from oracle.adjoint import EulerianStep  # noqa: E402
from oracle.scheme import Config as OConfig  # noqa: E402
from oracle.scheme import GTSSolver  # noqa: E402
from workloads import vortex_case  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _solver(mesh, Q0, M, flux="rusanov"):
    from paper_1408_3719_amd import Config, Solver
    return Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0,
                  Config(M=M, levels=1, mesh_velocity="eulerian", flux=flux))


@pytest.mark.parametrize("name,M,flux", [c + ("rusanov",) for c in CASES] + [c + ("hll",) for c in HLL_CASES])
def test_adjoint_matches_reverse_mode_oracle(name, M, flux):
    mesh, Q0 = _case(name, M)
    print(f"adjoint {name} M={M} {flux} {mesh.n_elems} triangles", flush=True)
    cfg = OConfig(M=M, levels=1, mesh_velocity="eulerian", flux=flux)
    o = GTSSolver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
    dt = 0.5 * float(o.dtcfl.min())
    st = EulerianStep(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    rng = np.random.default_rng(1)
    qb = rng.standard_normal(Q0.shape)
    ref = st.vjp(Q0, dt, qb)
    g = _solver(mesh, Q0, M, flux)
    Qa, Xa, _ = g.download()
    out = g.adjoint_gts_step(dt, qb).cpu().numpy().T
    for v in range(4):
        err = np.abs(out[:, v] - ref[:, v]).max() / np.abs(ref[:, v]).max()
        assert err < TOL, (v, err)
    # the simulation state is untouched, and the step it differentiates is the forward one
    Qb, Xb, _ = g.download()
    assert np.array_equal(Qa, Qb) and np.array_equal(Xa, Xb)
    g.step_gts(dt, 1)
    Q1, X1, _ = g.download()
    assert np.array_equal(X1, Xa)
    q1 = st.step(Q0, dt)
    assert np.abs(Q1 - q1).max() <= TOL * np.abs(q1).max()


def test_adjoint_after_steps_and_repeated_calls():
    """From a state reached by forward steps; two calls in a row agree and the
    output buffer of the first is not touched by the second."""
    mesh, Q0 = _case("vortex", 2)
    g = _solver(mesh, Q0, 2)
    g.step_gts(10.0, 3)
    Q, _, _ = g.download()
    cfg = OConfig(M=2, levels=1, mesh_velocity="eulerian")
    o = GTSSolver(mesh.nodes, mesh.tris, Q, cfg, bedges=mesh.bedges)
    dt = 0.5 * float(o.dtcfl.min())
    st = EulerianStep(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    rng = np.random.default_rng(2)
    qb = rng.standard_normal(Q.shape)
    a = g.adjoint_gts_step(dt, qb)
    b = g.adjoint_gts_step(dt, 2.0 * qb)
    ref = st.vjp(Q, dt, qb)
    a = a.cpu().numpy().T
    b = b.cpu().numpy().T
    assert np.abs(a - ref).max() < TOL * np.abs(ref).max()
    assert np.abs(b - 2.0 * a).max() < 1e-13 * np.abs(b).max()      # linear in qbar_next


def test_adjoint_rejects_unsupported_modes():
    from paper_1408_3719_amd import Config, Solver
    from paper_1408_3719_amd._lib import AderError
    mesh, Q0 = _case("vortex", 2)
    lag = Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=2, levels=1))
    with pytest.raises(AderError):
        lag.adjoint_gts_step(1e-3, np.zeros_like(Q0))
    osh = Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0,
                 Config(M=2, levels=1, mesh_velocity="eulerian", flux="osher"))   # not covered
    with pytest.raises(AderError):
        osh.adjoint_gts_step(1e-3, np.zeros_like(Q0))
    e = _solver(mesh, Q0, 2)
    with pytest.raises(AderError):
        e.adjoint_gts_step(-1.0, np.zeros_like(Q0))
    e.debug_macro_begin(10.0, 1)          # a macro step in progress
    with pytest.raises(AderError):
        e.adjoint_gts_step(1e-3, np.zeros_like(Q0))


def test_adjoint_full_size_against_gpu_differences_and_conservation():
    """80k-triangle vortex, M=2: <Qbar, (F(Q+hv) - F(Q-hv)) / 2h> of the GPU
    forward step against <adjoint(Qbar), v>, and the adjoint of the conserved
    totals equal to the element areas away from the boundary."""
    import torch
    mesh, Q0 = vortex_case(80_000, seed=1)
    rng = np.random.default_rng(5)
    # the vortex's far field is uniform to ~1e-7, where the WENO indicators sit
    # near eps and no difference quotient is linear; a 1e-3 perturbation keeps
    # every indicator well above eps
    Q0 = Q0 * (1.0 + 1e-3 * rng.standard_normal(Q0.shape))
    print(f"adjoint full size: {mesh.n_elems} triangles", flush=True)
    g = _solver(mesh, Q0, 2)
    dt = 0.5 * float(g.dump("DTCFL").min())
    NE = mesh.n_elems
    qb = rng.standard_normal(Q0.shape)
    ad_vec = g.adjoint_gts_step(dt, qb).cpu().numpy().T
    torch.cuda.synchronize()

    def F(Q):
        g.upload_state(Q, 0.0)
        st = g.step_gts(dt, 1)
        assert st["t"] == dt
        return g.download()[0]

    h = 1e-8
    for k in range(2):
        v = rng.standard_normal(Q0.shape) * np.abs(Q0).max(axis=0)
        fd = ((F(Q0 + h * v) - F(Q0 - h * v)) * qb).sum() / (2 * h)
        ad = (ad_vec * v).sum()
        print(f"direction {k}: fd {fd:.12e} adjoint {ad:.12e}", flush=True)
        assert abs(fd - ad) <= 1e-6 * np.abs(ad_vec * v).sum(), (k, fd, ad)
    # conservation identity
    g.upload_state(Q0, 0.0)
    p = mesh.nodes[mesh.tris]
    A = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
               - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    edges = g.dump("TOPO_EDGES")                  # a, b, L, R, el, er
    sten = g.dump("TOPO_STENCILS")
    bnd = np.unique(edges[edges[:, 3] < 0, 2])
    reach = np.zeros(NE, bool)
    for i in bnd:
        s = sten[i]
        reach[s[s >= 0]] = True
    far = ~reach
    for var in range(4):
        q = np.zeros((NE, 4))
        q[:, var] = A
        out = g.adjoint_gts_step(dt, q).cpu().numpy().T
        exp = np.zeros((NE, 4))
        exp[:, var] = A
        assert np.abs(out[far] - exp[far]).max() <= 1e-12 * A.max(), var


@pytest.mark.parametrize("every", [2, 10])
def test_trajectory_gradient_matches_oracle(every):
    """Gradient of a weighted sum of Q^5 with respect to Q^0 through five
    steps (torch.autograd.Function over the library's steps and adjoints,
    checkpoints every `every` steps) against autograd through five oracle
    steps."""
    import torch

    from paper_1408_3719_amd.trajectory import gts_trajectory
    mesh, Q0 = _case("vortex", 2)
    cfg = OConfig(M=2, levels=1, mesh_velocity="eulerian")
    o = GTSSolver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
    dt = 0.4 * float(o.dtcfl.min())
    st = EulerianStep(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    rng = np.random.default_rng(7)
    W = rng.standard_normal(Q0.shape)
    q = torch.tensor(Q0, dtype=torch.float64, requires_grad=True)
    x = q
    for _ in range(5):
        x = st(x, dt)
    (x * torch.tensor(W)).sum().backward()
    ref_q5, ref_g = x.detach().numpy(), q.grad.numpy()

    g = _solver(mesh, Q0, 2)
    q0 = torch.tensor(Q0.T.copy(), dtype=torch.float64, device="cuda", requires_grad=True)
    q5 = gts_trajectory(g, q0, dt, 5, every=every)
    (q5 * torch.tensor(W.T.copy(), device="cuda")).sum().backward()
    got_q5 = q5.detach().cpu().numpy().T
    got_g = q0.grad.cpu().numpy().T
    assert np.abs(got_q5 - ref_q5).max() <= TOL * np.abs(ref_q5).max()
    for v in range(4):
        err = np.abs(got_g[:, v] - ref_g[:, v]).max() / np.abs(ref_g[:, v]).max()
        assert err < TOL, (v, err)


def test_explosion_100_steps_gradient_against_central_differences():
    """The adjoint workload: 50k-triangle explosion, M=2, 100 global steps on a
    fixed mesh with checkpoints every 10 steps; J = total energy inside r < 0.3
    at the final time; dJ/d(initial density) against central differences with
    h = 1e-6 on 32 seeded directions. The piecewise-constant data get the
    seeded 1e-3 perturbation that breaks exact ties (where differences see the
    mean of two subgradients)."""
    import torch

    from paper_1408_3719_amd.trajectory import gts_trajectory
    from workloads import explosion_case
    mesh, Q0 = explosion_case(50_000, seed=7)
    NE = mesh.n_elems
    rng = np.random.default_rng(11)
    Q0 = Q0 * (1.0 + 1e-3 * rng.standard_normal(Q0.shape))
    p = mesh.nodes[mesh.tris]
    A = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
               - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    c = p.mean(axis=1)
    W = np.zeros((4, NE))
    inner = np.hypot(c[:, 0], c[:, 1]) < 0.3
    W[3, inner] = A[inner]
    Wd = torch.tensor(W, device="cuda")
    s = _solver(mesh, Q0, 2)
    dt = 0.5 * float(s.dump("DTCFL").min())
    q0 = torch.tensor(Q0.T.copy(), device="cuda", requires_grad=True)
    (gts_trajectory(s, q0, dt, 100, every=10) * Wd).sum().backward()
    g = q0.grad[0].cpu().numpy()

    def J(Q):
        s.upload_state(Q, 0.0)
        for k in range(100):
            s.step_gts((k + 1) * dt, 1)
        return float((s.download_q() * Wd).sum())

    h = 1e-6
    worst = 0.0
    for d in range(32):
        v = np.zeros_like(Q0)
        v[:, 0] = rng.standard_normal(NE) * Q0[:, 0]
        fd = (J(Q0 + h * v) - J(Q0 - h * v)) / (2 * h)
        ad = float((g * v[:, 0]).sum())
        worst = max(worst, abs(fd - ad) / np.abs(g * v[:, 0]).sum())
    print(f"32 directions: worst |fd - adjoint| / sum|terms| = {worst:.2e}", flush=True)
    assert worst < 1e-5
