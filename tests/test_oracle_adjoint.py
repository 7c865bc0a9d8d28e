"""Pins of the reverse-mode oracle (oracle/adjoint.py): one global time step on
a fixed mesh, and one with the mesh moving with the fluid, with dt held fixed.  The torch forward map must equal the NumPy
oracle's step, its vector-Jacobian product must match central differences of
the NumPy oracle's step, and the adjoint of the conserved totals must be the
element areas wherever the boundary flux cannot reach (conservation of the
scheme, eq. PDEfinal)."""
import numpy as np
import pytest

from oracle.adjoint import EulerianStep
from oracle.scheme import Config, GTSSolver
from workloads import explosion_case, sod_case, vortex_case


def _case(name, M):
    if name == "vortex":
        return vortex_case(400, seed=5)
    rng = np.random.default_rng(3)
    mesh, Q0 = sod_case(300, seed=11) if name == "sod" else explosion_case(500, seed=7)
    # break the exact ties of the piecewise-constant data (max and |.| kinks)
    return mesh, Q0 * (1.0 + 1e-3 * rng.standard_normal(Q0.shape))


def _setup(name, M, flux="rusanov"):
    mesh, Q0 = _case(name, M)
    cfg = Config(M=M, levels=1, mesh_velocity="eulerian", flux=flux)
    o = GTSSolver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
    dt = 0.5 * float(o.dtcfl.min())
    st = EulerianStep(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    return mesh, Q0, cfg, o, dt, st


CASES = [("vortex", 1), ("vortex", 2), ("vortex", 3), ("sod", 1), ("sod", 2), ("explosion", 2)]
HLL_CASES = [("vortex", 2), ("sod", 2), ("explosion", 2)]


@pytest.mark.parametrize("name,M", CASES)
def test_forward_equals_numpy_step(name, M):
    mesh, Q0, cfg, o, dt, st = _setup(name, M)
    o.step(dt)                                 # dt below the CFL step: this is the step taken
    assert o.T == dt
    Q1 = st.step(Q0, dt)
    assert np.abs(Q1 - o.Q).max() <= 1e-14 * np.abs(o.Q).max()


@pytest.mark.parametrize("name,M", CASES)
def test_vjp_matches_central_differences(name, M):
    """<Qbar, (F(Q+hv) - F(Q-hv)) / 2h> of the NumPy step against <vjp(Qbar), v>;
    h is relative to the data's scale and small enough for the steep WENO
    weights at the jumps (the error falls as h^2 down to ~1e-7 of the terms)."""
    mesh, Q0, cfg, o, dt, st = _setup(name, M)
    rng = np.random.default_rng(0)
    qb = rng.standard_normal(Q0.shape)
    g = st.vjp(Q0, dt, qb)

    def F(Q):
        s = GTSSolver(mesh.nodes, mesh.tris, Q, cfg, bedges=mesh.bedges, topo=o.topo)
        s.step(dt)
        return s.Q

    h = 1e-8
    for k in range(2):
        v = rng.standard_normal(Q0.shape) * np.abs(Q0).max(axis=0)
        fd = ((F(Q0 + h * v) - F(Q0 - h * v)) * qb).sum() / (2 * h)
        ad = (g * v).sum()
        # relative to the size of the terms summed (they cancel strongly at jumps)
        assert abs(fd - ad) <= 1e-6 * np.abs(g * v).sum(), (k, fd, ad)


@pytest.mark.parametrize("name,M", [("vortex", 2), ("explosion", 2)])
def test_adjoint_of_conserved_totals_is_the_area(name, M):
    """sum_i |T_i| Q_i^{n+1} = sum_i |T_i| Q_i^n - boundary flux, so the adjoint
    of Qbar_i = |T_i| e_v is |T_j| e_v for every element j whose average cannot
    reach a boundary flux (outside the stencils of the boundary elements)."""
    mesh, Q0, cfg, o, dt, st = _setup(name, M)
    topo = o.topo
    bnd = np.unique(topo.edge_elems[topo.edge_elems[:, 1] < 0, 0])
    reach = np.zeros(topo.n_elems, bool)
    for i in bnd:
        s = topo.stencils[i]
        reach[s[s >= 0]] = True
    far = ~reach
    assert far.sum() > 0.3 * topo.n_elems
    for var in range(4):
        qb = np.zeros_like(Q0)
        qb[:, var] = st.area
        g = st.vjp(Q0, dt, qb)
        exp = np.zeros_like(Q0)
        exp[:, var] = st.area
        assert np.abs(g[far] - exp[far]).max() <= 1e-12 * st.area.max(), var
        # and the boundary does act on the rest (the pin is not vacuous)
        if var in (1, 2):
            assert np.abs(g[reach] - exp[reach]).max() > 1e-8 * st.area.max()


@pytest.mark.parametrize("name,M", HLL_CASES)
def test_hll_forward_and_vjp(name, M):
    """The same two pins with the HLL flux."""
    mesh, Q0, cfg, o, dt, st = _setup(name, M, flux="hll")
    o.step(dt)
    assert np.abs(st.step(Q0, dt) - o.Q).max() <= 1e-14 * np.abs(o.Q).max()
    rng = np.random.default_rng(0)
    qb = rng.standard_normal(Q0.shape)
    g = st.vjp(Q0, dt, qb)

    def F(Q):
        s = GTSSolver(mesh.nodes, mesh.tris, Q, cfg, bedges=mesh.bedges, topo=o.topo)
        s.step(dt)
        return s.Q

    h = 1e-8
    v = rng.standard_normal(Q0.shape) * np.abs(Q0).max(axis=0)
    fd = ((F(Q0 + h * v) - F(Q0 - h * v)) * qb).sum() / (2 * h)
    ad = (g * v).sum()
    assert abs(fd - ad) <= 1e-6 * np.abs(g * v).sum(), (fd, ad)


# ---------------------------------------------------------------------------
# Lagrangian step: (Q, X) -> (Q', X'), the mesh moving with the fluid
# ---------------------------------------------------------------------------
def _setup_lagrangian(name, M, flux="rusanov"):
    from oracle.adjoint import LagrangianStep
    mesh, Q0 = _case(name, M)
    cfg = Config(M=M, levels=1, mesh_velocity="lagrangian", flux=flux)
    o = GTSSolver(mesh.nodes, mesh.tris, Q0, cfg, bedges=mesh.bedges)
    dt = 0.5 * float(o.dtcfl.min())
    st = LagrangianStep(mesh.nodes, mesh.tris, cfg, bedges=mesh.bedges, topo=o.topo)
    return mesh, Q0, cfg, o, dt, st


LAGR_CASES = [("vortex", 1), ("vortex", 2), ("vortex", 3), ("sod", 2), ("explosion", 2)]


@pytest.mark.parametrize("name,M", LAGR_CASES)
def test_lagrangian_forward_equals_numpy_step(name, M):
    """The torch Lagrangian step (reconstruction on the moving geometry,
    predictor with the mesh ODE, node solver, moving patches, new areas)
    equals the NumPy oracle's global step: averages and node positions."""
    mesh, Q0, cfg, o, dt, st = _setup_lagrangian(name, M)
    Q1, X1 = st.step(Q0, mesh.nodes, dt)
    o.step(dt)
    assert o.T == dt
    assert np.abs(Q1 - o.Q).max() <= 1e-14 * np.abs(o.Q).max()
    assert np.abs(X1 - o.X).max() <= 1e-14 * np.abs(o.X).max()
    assert np.abs(X1 - mesh.nodes).max() > 1e-6 * np.ptp(mesh.nodes)       # the mesh moved


@pytest.mark.parametrize("name,M", [("vortex", 1), ("vortex", 2), ("explosion", 2)])
def test_lagrangian_vjp_matches_central_differences(name, M):
    """<(Qbar, Xbar), (F(Q+hv, X+hy) - F(Q-hv, X-hy)) / 2h> of the NumPy step
    (topology held) against the vector-Jacobian product, with directions in
    both the averages and the node positions, and in each alone."""
    mesh, Q0, cfg, o, dt, st = _setup_lagrangian(name, M)
    rng = np.random.default_rng(1)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    gq, gx = st.vjp(Q0, mesh.nodes, dt, qb, xb)

    def F(Q, X):
        s = GTSSolver(X, mesh.tris, Q, cfg, bedges=mesh.bedges, topo=o.topo)
        s.step(dt)
        return s.Q, s.X

    h = 1e-8
    hx = h * np.ptp(mesh.nodes) * 1e-1
    for k, (wq, wx) in enumerate(((1, 1), (1, 0), (0, 1))):
        v = wq * rng.standard_normal(Q0.shape) * np.abs(Q0).max(axis=0)
        y = wx * rng.standard_normal(mesh.nodes.shape) * hx / h
        Qp, Xp = F(Q0 + h * v, mesh.nodes + h * y)
        Qm, Xm = F(Q0 - h * v, mesh.nodes - h * y)
        fd = (((Qp - Qm) * qb).sum() + ((Xp - Xm) * xb).sum()) / (2 * h)
        ad = (gq * v).sum() + (gx * y).sum()
        scale = np.abs(gq * v).sum() + np.abs(gx * y).sum()
        assert abs(fd - ad) <= 1e-6 * scale, (k, fd, ad)


@pytest.mark.parametrize("name,M", [("vortex", 2), ("explosion", 2)])
def test_lagrangian_adjoint_of_a_translation(name, M):
    """Moving every node by the same vector c leaves the averages unchanged and
    moves every new node by c (translation invariance of the scheme), so for
    any (Qbar, Xbar) the node-position adjoints sum to the sum of Xbar."""
    mesh, Q0, cfg, o, dt, st = _setup_lagrangian(name, M)
    rng = np.random.default_rng(2)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    _, gx = st.vjp(Q0, mesh.nodes, dt, qb, xb)
    scale = np.abs(gx).sum(axis=0)
    assert np.abs(gx.sum(axis=0) - xb.sum(axis=0)).max() <= 1e-12 * scale.max()
    assert np.abs(gx - xb).max() > 1e-3 * np.abs(xb).max()        # the geometry does act


@pytest.mark.parametrize("name,M", [("sod", 2), ("vortex", 2), ("explosion", 2)])
def test_lagrangian_hll_forward_equals_numpy_step(name, M):
    """The Lagrangian step with the HLL flux equals the NumPy global step
    (averages and positions)."""
    mesh, Q0, cfg, o, dt, st = _setup_lagrangian(name, M, flux="hll")
    Q1, X1 = st.step(Q0, mesh.nodes, dt)
    o.step(dt)
    assert np.abs(Q1 - o.Q).max() <= 1e-14 * np.abs(o.Q).max()
    assert np.abs(X1 - o.X).max() <= 1e-14 * np.abs(o.X).max()


@pytest.mark.parametrize("name,M", [("vortex", 2), ("explosion", 2)])
def test_lagrangian_hll_vjp_matches_central_differences(name, M):
    """The product of the Lagrangian HLL step against central differences of
    the NumPy step, directions in the averages and the node positions
    together. (The shock tube starts at rest: the wall's mirrored states then
    tie exactly in the HLL speed comparisons, where differences see the mean
    of two one-sided derivatives.)"""
    mesh, Q0, cfg, o, dt, st = _setup_lagrangian(name, M, flux="hll")
    rng = np.random.default_rng(3)
    qb = rng.standard_normal(Q0.shape)
    xb = rng.standard_normal(mesh.nodes.shape)
    gq, gx = st.vjp(Q0, mesh.nodes, dt, qb, xb)

    def F(Q, X):
        s = GTSSolver(X, mesh.tris, Q, cfg, bedges=mesh.bedges, topo=o.topo)
        s.step(dt)
        return s.Q, s.X

    h = 1e-8
    v = rng.standard_normal(Q0.shape) * np.abs(Q0).max(axis=0)
    y = rng.standard_normal(mesh.nodes.shape) * np.ptp(mesh.nodes) * 1e-1
    Qp, Xp = F(Q0 + h * v, mesh.nodes + h * y)
    Qm, Xm = F(Q0 - h * v, mesh.nodes - h * y)
    fd = (((Qp - Qm) * qb).sum() + ((Xp - Xm) * xb).sum()) / (2 * h)
    ad = (gq * v).sum() + (gx * y).sum()
    assert abs(fd - ad) <= 1e-6 * (np.abs(gq * v).sum() + np.abs(gx * y).sum()), (fd, ad)
