"""Pins of the oracle's per-element numerics against exact solutions."""
import math

import numpy as np
import pytest

from oracle import euler
from oracle import tables as tb
from oracle.scheme import (Config, affine_map, node_velocity, patch_batch, predictor_batch,
                           reconstruct_batch, rusanov_flux, tri_area)
from oracle.topology import build_topology
from workloads import strip_mesh

GAMMA = 1.4


def _poly(M, seed, nvar=4):
    rng = np.random.default_rng(seed)
    mons = tb.monomials(M)
    C = rng.normal(size=(nvar, len(mons)))
    C[:, 0] += 3.0

    def p(x, y):
        return np.stack([sum(c[k] * x ** a * y ** b for k, (a, b) in enumerate(mons)) for c in C], -1)
    return p


def _exact_means(X, p, n=6):
    """Means of p over triangles X (..., 3, 2) with a Duffy rule exact far beyond M."""
    xi, eta, w = tb.duffy_rule(n)
    x = affine_map(X, xi, eta)
    return np.einsum("...qv,q->...v", p(x[..., 0], x[..., 1]), w / w.sum())


@pytest.fixture(scope="module")
def small_mesh():
    return strip_mesh(0.0, 1.0, 0.0, 1.0, 0.09, seed=5)


@pytest.mark.parametrize("M", [1, 2, 3])
@pytest.mark.parametrize("virtual", [False, True])
def test_reconstruction_reproduces_polynomials(small_mesh, M, virtual):
    """Every stencil reproduces a degree-M polynomial exactly, hence so does any
    WENO combination (eqs. intConsRec, eqn.weno), also on moved (virtual) stencils."""
    topo = build_topology(small_mesh.nodes, small_mesh.tris, M)
    X = small_mesh.nodes[small_mesh.tris]
    elems = np.arange(topo.n_elems)
    sten = topo.stencils
    valid = sten[:, :, 0] >= 0
    ss = np.where(sten >= 0, sten, elems[:, None, None])
    Xs = X[ss].copy()
    if virtual:
        rng = np.random.default_rng(11)
        pert = 0.15 * 0.09 * rng.normal(size=Xs.shape)
        pert[:, :, 0] = 0.0           # element i keeps its real geometry
        Xs = Xs + pert
    p = _poly(M, 3)
    Qs = _exact_means(Xs, p)
    Qi = _exact_means(X, p)
    cfg = Config(M=M)
    wnod, _, what_s, omega = reconstruct_batch(M, cfg, X, Qi, Xs, Qs, valid)
    nodes = tb.nodal_xy(M)
    xn = affine_map(X, nodes[:, 0], nodes[:, 1])
    exact = p(xn[..., 0], xn[..., 1])
    err = np.abs(wnod - exact).max() / np.abs(exact).max()
    assert err < 1e-10, err
    assert valid[:, 0].all()
    assert valid.sum() > 3 * topo.n_elems     # most sector stencils exist
    assert np.allclose(omega.sum(axis=1), 1.0)


@pytest.mark.parametrize("M", [1, 2])
def test_weno_linear_weights_for_constant_data(small_mesh, M):
    topo = build_topology(small_mesh.nodes, small_mesh.tris, M)
    X = small_mesh.nodes[small_mesh.tris]
    elems = np.arange(topo.n_elems)
    valid = topo.stencils[:, :, 0] >= 0
    ss = np.where(topo.stencils >= 0, topo.stencils, elems[:, None, None])
    Q = np.tile([1.0, 0.2, -0.3, 2.5], (topo.n_elems, 1))
    cfg = Config(M=M)
    wnod, _, _, omega = reconstruct_batch(M, cfg, X, Q, X[ss], Q[ss], valid)
    lam = np.where(np.arange(7) == 0, cfg.weno_lambda, 1.0)
    lin = np.where(valid, lam, 0.0)
    lin = lin / lin.sum(axis=1, keepdims=True)
    assert np.allclose(omega, lin[:, :, None], rtol=1e-12)
    assert np.abs(wnod - Q[:, None, :]).max() < 1e-13


def _one_triangle():
    return np.array([[[0.1, 0.2], [0.37, 0.25], [0.18, 0.46]]])


@pytest.mark.parametrize("M", [1, 2, 3])
@pytest.mark.parametrize("mode", ["eulerian", "lagrangian"])
def test_predictor_keeps_constant_state(M, mode):
    Q = np.array([1.3, 0.4, -0.2, 3.1])
    nb = tb.sizes(M)["nb"]
    cfg = Config(M=M, mesh_velocity=mode)
    out = predictor_batch(M, cfg, np.tile(Q, (1, nb, 1)), _one_triangle(), np.array([0.01]))
    assert np.abs(out["q"] - Q).max() < 1e-14
    assert np.abs(out["avg"] - Q).max() < 1e-14
    assert np.abs(out["trace"] - Q).max() < 1e-14


@pytest.mark.parametrize("M", [1, 2, 3])
def test_predictor_entropy_wave_eulerian(M):
    """Uniform u, v, p and a degree-M density: every flux is in the space, the
    space-time solution rho(x - u t) is in P_M x P_M and M+1 Picard sweeps
    reproduce it at all nodes (eqs. PDECG..CGfinal)."""
    u, v, p0 = 0.7, -0.4, 1.0
    prho = _poly(M, 7, nvar=1)

    def rho(x, y):
        return 2.0 + 0.3 * prho(x, y)[..., 0]

    def cons(x, y):
        r = rho(x, y)
        return np.stack([r, r * u, r * v, p0 / (GAMMA - 1) + 0.5 * r * (u * u + v * v)], -1)

    X = _one_triangle()
    nodes = tb.nodal_xy(M)
    xn = affine_map(X, nodes[:, 0], nodes[:, 1])[0]
    dt = 0.05
    cfg = Config(M=M, mesh_velocity="eulerian")
    out = predictor_batch(M, cfg, cons(xn[:, 0], xn[:, 1])[None], X, np.array([dt]))
    tn = tb.time_nodes(M)
    exp = np.stack([cons(xn[:, 0] - u * t * dt, xn[:, 1] - v * t * dt) for t in tn], axis=1)
    assert np.abs(out["q"][0] - exp).max() < 1e-12


@pytest.mark.parametrize("M", [1, 2, 3])
def test_predictor_entropy_wave_lagrangian(M):
    """With V = v uniform the mesh translates exactly and the density carried
    by the moving nodes stays constant in time."""
    u, v, p0 = 0.7, -0.4, 1.0
    prho = _poly(M, 8, nvar=1)
    X = _one_triangle()
    nodes = tb.nodal_xy(M)
    xn = affine_map(X, nodes[:, 0], nodes[:, 1])[0]
    r = 2.0 + 0.3 * prho(xn[:, 0], xn[:, 1])[..., 0]
    w = np.stack([r, r * u, r * v, p0 / (GAMMA - 1) + 0.5 * r * (u * u + v * v)], -1)
    dt = 0.05
    out = predictor_batch(M, Config(M=M), w[None], X, np.array([dt]))
    tn = tb.time_nodes(M)
    assert np.abs(out["q"][0] - w[:, None, :]).max() < 1e-12
    xexp = xn[:, None, :] + np.array([u, v]) * (tn * dt)[None, :, None]
    assert np.abs(out["x"][0] - xexp).max() < 1e-14
    assert np.allclose(out["vvel"][0], np.array([u, v]), atol=1e-14)


def test_node_solver_uniform_velocity():
    """eqs. eqnNScs/NodesVel: uniform vertex velocities average to themselves."""
    rng = np.random.default_rng(1)
    for M in (1, 2, 3):
        R = 6
        vv = np.tile(np.array([0.3, -1.1]), (R, M + 1, 1))
        t0 = rng.uniform(0, 0.5, R)
        t1 = t0 + rng.uniform(0.1, 0.5, R)
        V = node_velocity(M, vv, t0, t1, rng.uniform(0.5, 2, R))
        assert np.allclose(V, [0.3, -1.1], atol=1e-15)


def _patch(P, ticks, trL, trR=None, M=1):
    E = P.shape[0]
    one = np.ones(E, np.int64)
    zero = np.zeros(E, np.int64)
    hasR = np.zeros(E, bool) if trR is None else np.ones(E, bool)
    trR = trL if trR is None else trR
    return patch_batch(M, Config(M=M), P, ticks, zero, one * 4, trL, zero, one * 4, trR, hasR,
                       avgL=trL[:, 0])    # constant traces: the means equal them


def _const_trace(Q, M, E=1):
    return np.tile(Q, (E, M + 1, M + 1, 1))


def test_patch_static_and_translating_edge():
    a = np.array([0.2, 0.1])
    b = np.array([0.5, 0.4])
    dt = 0.3
    Q = np.array([1.0, 0.1, 0.2, 2.5])
    P = np.array([[[*a, 0], [*b, 0], [*b, dt], [*a, dt]]])
    ticks = np.array([[0.0, 0.0, 4.0, 4.0]])
    _, Nint = _patch(P, ticks, _const_trace(Q, 1))
    d = b - a
    assert np.allclose(Nint[0], [dt * d[1], -dt * d[0], 0.0], atol=1e-16)
    V = np.array([0.7, -0.2])
    P = np.array([[[*a, 0], [*b, 0], [*(b + V * dt), dt], [*(a + V * dt), dt]]])
    G, Nint = _patch(P, ticks, _const_trace(Q, 1))
    n = np.array([d[1], -d[0]])
    assert np.allclose(Nint[0], [dt * n[0], dt * n[1], -dt * V @ n], atol=1e-15)
    # consistency: equal states give the physical flux through the normal
    Ft = euler.flux_f(Q, GAMMA) * Nint[0, 0] + euler.flux_g(Q, GAMMA) * Nint[0, 1] + Q * Nint[0, 2]
    assert np.allclose(G[0], Ft, atol=1e-15)


def test_patches_close_space_time_volume_with_hanging_nodes():
    """eq. eqn.gcl: the lateral patches of a triangle swept in several partial
    moves (hanging nodes in time) plus bottom and top close the volume."""
    rng = np.random.default_rng(3)
    X0 = np.array([[0.0, 0.0], [1.0, 0.1], [0.3, 0.9]])
    d = 0.25
    # node k positions/ticks over three partial moves: node 0 moves 0->1, node 1 0->2, then all to 4
    Xs = [X0.copy()]
    T = [np.zeros(3)]
    moves = [({0}, 1), ({1}, 2), ({0, 1, 2}, 4)]
    total = np.zeros(3)
    for nodes, tick in moves:
        Xn, Tn = Xs[-1].copy(), T[-1].copy()
        for k in nodes:
            Xn[k] = Xn[k] + 0.05 * rng.normal(size=2)
            Tn[k] = tick
        for k in range(3):
            a, b = k, (k + 1) % 3
            if a in nodes or b in nodes:
                P = np.array([[[*Xs[-1][a], T[-1][a] * d], [*Xs[-1][b], T[-1][b] * d],
                               [*Xn[b], Tn[b] * d], [*Xn[a], Tn[a] * d]]])
                ticks = np.array([[T[-1][a], T[-1][b], Tn[b], Tn[a]]])
                _, Nint = _patch(P, ticks, _const_trace(np.array([1, 0, 0, 2.5]), 1))
                total += Nint[0]
        Xs.append(Xn)
        T.append(Tn)
    A0 = tri_area(X0)
    A1 = tri_area(Xs[-1])
    total += np.array([0, 0, A1 - A0])
    assert np.abs(total).max() < 1e-15


def test_rusanov_reduces_to_eulerian_flux():
    rng = np.random.default_rng(2)
    ql = np.array([1.0, 0.3, -0.1, 2.6])
    qr = np.array([0.5, -0.2, 0.1, 1.4])
    n = np.array([0.6, 0.8])
    F = rusanov_flux(ql, qr, np.array([n[0], n[1], 0.0]), GAMMA)

    def fn(q):
        return euler.flux_f(q, GAMMA) * n[0] + euler.flux_g(q, GAMMA) * n[1]

    def sp(q):
        r, u, v, p = euler.primitives(q, GAMMA)
        return abs(u * n[0] + v * n[1]) + math.sqrt(GAMMA * p / r)

    exp = 0.5 * (fn(ql) + fn(qr)) - 0.5 * max(sp(ql), sp(qr)) * (qr - ql)
    assert np.allclose(F, exp, atol=1e-15)
    # moving face: the ALE flux sees the relative normal velocity
    N = np.array([n[0], n[1], -0.3])
    F2 = rusanov_flux(ql, ql, N, GAMMA)
    assert np.allclose(F2, fn(ql) - 0.3 * ql, atol=1e-15)


def test_slip_wall_carries_no_mass_or_energy_flux():
    """A static slip wall (mirror state) passes only the pressure force, also
    when the same batch holds interior edges."""
    M = 1
    Q = np.array([1.3, 0.4, -0.7, 3.1])
    dt = 0.2
    a, b = np.array([0.0, 0.0]), np.array([1.0, 0.0])
    P = np.array([[[*a, 0], [*b, 0], [*b, dt], [*a, dt]]] * 2)
    ticks = np.tile([0.0, 0.0, 4.0, 4.0], (2, 1))
    tr = _const_trace(Q, M, E=2)
    one = np.ones(2, np.int64) * 4
    zero = np.zeros(2, np.int64)
    hasR = np.array([False, True])
    bc = np.array([2, 0])
    G, Nint = patch_batch(M, Config(M=M), P, ticks, zero, one, tr, zero, one, tr, hasR, bc)
    p = (GAMMA - 1) * (Q[3] - 0.5 * (Q[1] ** 2 + Q[2] ** 2) / Q[0])
    assert abs(G[0, 0]) < 1e-15 and abs(G[0, 3]) < 1e-15          # no mass, no work
    assert abs(G[0, 1]) < 1e-15                                    # no tangential force
    assert G[0, 2] / Nint[0, 1] > p                                # pressure plus impact
    assert abs(G[1, 0] - Q[2] * Nint[1, 1]) < 1e-15                # interior edge unaffected
