"""Parity at workload size: the first cycle of the 80k-triangle vortex (M=2,
3 levels) element by element with launches one by one; the explosion with 4
levels at 30k triangles over two macro steps in the launch configuration the
benchmark times (autotuned settings, captured graphs) and with persistent
grids that stride the active list; the explosion at its full 400k triangles
on sampled elements, at t = 0 and in a cycle in the middle of the run, and the
timed configuration bit-identical to launches one by one there."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from test_gpu_parity import TOL, _gpu_solver, _oracle, _span, rel, rel_groups  # noqa: E402

from workloads import explosion_case, vortex_case  # noqa: E402

pytestmark = pytest.mark.gpu


def test_bench_configuration_first_cycle_parity():
    mesh, Q0 = vortex_case(80_000, seed=1)
    print(f"vortex mesh {mesh.n_elems} triangles", flush=True)
    g = _gpu_solver(mesh, Q0, 2, 3)
    o = _oracle(mesh, Q0, 2, 3)
    assert rel(np.transpose(g.dump("WNOD"), (2, 0, 1)), o.st.wnod) < TOL
    assert rel(g.dump("DTCFL"), o.st.dtcfl) < TOL
    g.debug_macro_begin(1.0, 3)
    o.macro_begin(1.0)
    assert np.array_equal(g.dump("STEP"), o.st.s)
    assert rel(np.moveaxis(g.dump("TRACE"), -1, 0), o.st.trace) < TOL
    assert len(np.unique(o.st.s)) == 3                  # all three levels in use
    o.cycle()
    g.debug_cycles(1)
    assert np.array_equal(g.dump("TICK"), o.st.n)
    assert np.array_equal(g.dump("STEP"), o.st.s)
    assert np.array_equal(g.dump("NTICK"), o.st.nk)
    assert (rel_groups(g.dump("Q").T, o.st.Q) < TOL).all()
    assert np.abs(g.dump("X").T - o.st.X).max() < TOL * _span(mesh)
    assert rel(np.transpose(g.dump("WNOD"), (2, 0, 1)), o.st.wnod) < TOL
    live = o.st.s > 0
    assert rel(np.moveaxis(g.dump("TRACE"), -1, 0)[live], o.st.trace[live]) < TOL


def test_explosion_timed_configuration_parity():
    """Explosion, 30k triangles, M=2, 4 levels, two macro steps against the
    oracle in three launch configurations: the one bench.py times (settings
    picked by the autotuner, each macro step replayed from its captured graph),
    persistent grids of one workgroup per CU striding the active and predictor
    lists several times per launch (the striding loops of the reconstruction
    and predictor kernels), and every kernel launched one by one with default
    settings. The three are bit-identical to each other."""
    mesh, Q0 = explosion_case(30_000, seed=7)
    print(f"explosion mesh {mesh.n_elems} triangles", flush=True)
    o = _oracle(mesh, Q0, 2, 4)
    o.run(1.0, max_macro_steps=2)
    # one pass of a persistent grid of 256 workgroups covers 256 * 32
    # reconstructions and 256 * 40 predictors at M=2; the lists are longer
    print(f"oracle: {o.st.cycles} cycles, largest active set {max(o.st.active_sizes)}", flush=True)
    assert max(o.st.active_sizes) > 256 * 40 * 1.2, max(o.st.active_sizes)
    tuned = _gpu_solver(mesh, Q0, 2, 4)
    choice = tuned.autotune(2)
    print("autotuned", choice, flush=True)
    stride = _gpu_solver(mesh, Q0, 2, 4)
    stride.set_tune(sched_chunk=choice["sched_chunk"], list_wg_per_cu=1)
    eager = _gpu_solver(mesh, Q0, 2, 4)
    eager.set_graphs(False)
    out = []
    for name, g in (("tuned", tuned), ("stride", stride), ("eager", eager)):
        st = g.step_lts(1.0, 2)
        Q, X, t = g.download()
        print(f"{name}: updates {st['element_updates']} (oracle {o.st.updates}) "
              f"extra cycles {st['extra_cycles']}", flush=True)
        assert st["element_updates"] == o.st.updates, name
        assert st["node_moves"] == o.st.node_moves and st["patches"] == o.st.patches, name
        assert st["cfl_overshoots"] == 0
        assert (rel_groups(Q, o.st.Q) < TOL).all(), name
        assert np.abs(X - o.st.X).max() < TOL * _span(mesh), name
        out.append((Q, X, t))
    for Q, X, t in out[1:]:
        assert np.array_equal(Q, out[0][0]) and np.array_equal(X, out[0][1]) and np.array_equal(t, out[0][2])
    assert o.st.updates < 2 * 8 * mesh.n_elems         # fewer updates than GTS at the finest step


def test_explosion_full_size_sampled_parity_and_conservation():
    """The explosion workload at its full size (400k triangles, M=2, 4 levels):
    the pre-processing reconstruction and the macro-step start (predictor)
    element by element on a seeded sample of 2,000 elements, each computed by
    the oracle from its own stencil; CFL steps and levels on every element.
    Then two macro steps (16 cycles): mass, momentum and energy conserved to
    round-off (no wave reaches the boundary yet, and the uniform boundary
    pressure sums to zero force over the closed polygon), the GCL held, and
    fewer element updates than global steps at the finest step."""
    from oracle.scheme import Config as OConfig
    from oracle.scheme import (MACRO_TICKS, cfl_time_steps, level_step, macro_tick, predictor_batch,
                               reconstruct_batch)
    from oracle.topology import face_neighbours, stencils_of
    mesh, Q0 = explosion_case(400_000, seed=7)
    NE = mesh.n_elems
    print(f"explosion mesh {NE} triangles", flush=True)
    cfg = OConfig(M=2, levels=4)
    g = _gpu_solver(mesh, Q0, 2, 4)
    rng = np.random.default_rng(400)
    sample = np.sort(rng.choice(NE, 2000, replace=False))
    Xe = mesh.nodes[mesh.tris]
    sten = stencils_of(mesh.nodes, mesh.tris, 2, sample)
    valid = sten[:, :, 0] >= 0
    ss = np.where(sten >= 0, sten, sample[:, None, None])
    wnod_o, _, _, _ = reconstruct_batch(2, cfg, Xe[sample], Q0[sample], Xe[ss], Q0[ss], valid)
    assert rel(np.transpose(g.dump("WNOD"), (2, 0, 1))[sample], wnod_o) < TOL
    dt_o = cfl_time_steps(Xe, Q0, face_neighbours(mesh.tris), cfg.gamma, cfg.cfl)
    assert rel(g.dump("DTCFL"), dt_o) < TOL
    print("pre-processing checked", flush=True)
    g.debug_macro_begin(1.0, 4)
    delta = macro_tick(4, float(dt_o.min()), 0.0, 1.0, cfg.lts_fraction)
    assert abs(g.dump("SCAL")[1] - delta) <= 1e-14 * delta
    # the oracle's level rule at tick 0, on all elements at once (checked
    # against the rule itself on the sample)
    steps_o = np.full(NE, MACRO_TICKS, np.int64)
    while True:
        big = (steps_o > 1) & (steps_o * delta > dt_o)
        if not big.any():
            break
        steps_o[big] //= 2
    assert all(level_step(dt_o[i], delta, MACRO_TICKS, 0, False)[0] == steps_o[i] for i in sample)
    assert np.array_equal(g.dump("STEP"), steps_o)
    assert len(np.unique(steps_o)) == 4                 # all four levels in use
    pr = predictor_batch(2, cfg, wnod_o, Xe[sample], steps_o[sample] * delta, np.zeros(sample.size))
    assert rel(np.moveaxis(g.dump("TRACE"), -1, 0)[sample], pr["trace"]) < TOL
    assert rel(np.moveaxis(g.dump("VVEL"), -1, 0)[sample], pr["vvel"]) < TOL
    print("macro begin checked", flush=True)
    g.upload_state(Q0, 0.0)
    st = g.step_lts(1.0, 2)
    Q, X, _ = g.download()
    p = X[mesh.tris]
    A1 = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    A0 = 0.5 * ((Xe[:, 1, 0] - Xe[:, 0, 0]) * (Xe[:, 2, 1] - Xe[:, 0, 1])
                - (Xe[:, 2, 0] - Xe[:, 0, 0]) * (Xe[:, 1, 1] - Xe[:, 0, 1]))
    c0 = (A0[:, None] * Q0).sum(axis=0)
    c1 = (A1[:, None] * Q).sum(axis=0)
    scale = (A0[:, None] * np.abs(Q0)).sum(axis=0).max()
    print(f"two macro steps: t={st['t']:.3e} updates={st['element_updates']} drift={np.abs(c1 - c0) / scale}",
          flush=True)
    assert np.abs(c1 - c0).max() <= 1e-13 * scale
    assert st["max_gcl_residual"] < 1e-12
    assert st["element_updates"] < 2 * 8 * NE
    # the timed configuration at full size: persistent grids of one workgroup
    # per CU (the active lists are ~8x one pass, the node and edge sweeps
    # ~4x and ~18x), captured graphs, against default settings launched one
    # by one: bit-identical
    del g
    tg = _gpu_solver(mesh, Q0, 2, 4)
    tg.set_tune(sched_chunk=256, list_wg_per_cu=1, sweep_wg_per_cu=1)
    eg = _gpu_solver(mesh, Q0, 2, 4)
    eg.set_graphs(False)
    st_t, st_e = tg.step_lts(1.0, 2), eg.step_lts(1.0, 2)
    Qt, Xt, tt = tg.download()
    Qe, Xe2, te = eg.download()
    print(f"timed configuration: updates {st_t['element_updates']} / {st_e['element_updates']}", flush=True)
    assert st_t["element_updates"] == st_e["element_updates"] == st["element_updates"]
    assert np.array_equal(Qt, Qe) and np.array_equal(Xt, Xe2) and np.array_equal(tt, te)
    assert np.array_equal(Qe, Q) and np.array_equal(Xe2, X)


def test_explosion_full_size_mid_run_cycle_on_samples():
    """The explosion workload at its full size (400k triangles, M=2, 4 levels)
    in the middle of a run: one macro step, then the second macro step's
    start and three cycles; the fourth cycle is checked on seeded samples,
    each quantity recomputed by the oracle from the library's own state before
    (S0) or after (S1) the cycle: node motion of moved nodes over their own
    intervals (S0), the flux of every swept patch of elements not updated in
    the cycle through their memory variables (S0 and the new node positions),
    the reconstruction of updated elements from their stencils placed at their
    new tick (S1), and the new predictors (S1)."""
    from types import SimpleNamespace

    from oracle.scheme import Config as OConfig
    from oracle.scheme import (MACRO_TICKS, Solver, node_velocity, patch_batch, predictor_batch,
                               reconstruct_batch)
    from oracle.topology import build_edges, stencils_of
    mesh, Q0 = explosion_case(400_000, seed=7)
    NE, tris = mesh.n_elems, mesh.tris
    print(f"explosion mesh {NE} triangles", flush=True)
    cfg = OConfig(M=2, levels=4)
    g = _gpu_solver(mesh, Q0, 2, 4)
    g.step_lts(1.0, 1)
    g.debug_macro_begin(1.0, 4)
    g.debug_cycles(3)

    def state():
        return dict(Q=g.dump("Q").T.copy(), A=g.dump("A").copy(), Xe=g.dump("XE").T.reshape(NE, 3, 2).copy(),
                    n=g.dump("TICK").astype(np.int64), s=g.dump("STEP").astype(np.int64),
                    QM=g.dump("QM").T.copy(), wnod=np.transpose(g.dump("WNOD"), (2, 0, 1)).copy(),
                    avg=np.transpose(g.dump("AVG"), (2, 0, 1)).copy(),
                    trace=np.moveaxis(g.dump("TRACE"), -1, 0).copy(),
                    vvel=np.moveaxis(g.dump("VVEL"), -1, 0).copy(), X=g.dump("X").T.copy(),
                    nk=g.dump("NTICK").astype(np.int64))
    S0 = state()
    delta = float(g.dump("SCAL")[1])
    g.debug_cycles(1)
    S1 = state()
    rng = np.random.default_rng(404)
    act = np.nonzero(S1["n"] != S0["n"])[0]
    moved = np.nonzero(S1["nk"] != S0["nk"])[0]
    print(f"cycle: {act.size} updated, {moved.size} nodes moved", flush=True)
    assert act.size > 1000 and moved.size > 1000
    # node motion (eqs. eqn.dtau, NodesVel, eqnNScs, eqn.NScs.weights, eqn.newVertex)
    kk = np.sort(rng.choice(moved, 500, replace=False))
    dev = 0.0
    for k in kk:
        j, lv = np.nonzero(tris == k)
        tau0 = (S0["nk"][k] - S0["n"][j]) / S0["s"][j]
        tau1 = (S1["nk"][k] - S0["n"][j]) / S0["s"][j]
        V = node_velocity(2, S0["vvel"][j, lv], tau0, tau1, S0["Q"][j, 0] * S0["A"][j])
        x = S0["X"][k] + (S1["nk"][k] - S0["nk"][k]) * delta * V
        dev = max(dev, np.abs(x - S1["X"][k]).max())
    assert dev <= TOL * _span(mesh), dev
    # swept patches through the memory variables of elements not updated
    edge_nodes, edge_elems, edge_local, elem_edges = build_edges(tris)
    is_moved = S1["nk"] != S0["nk"]
    swept = is_moved[edge_nodes[:, 0]] | is_moved[edge_nodes[:, 1]]
    idle = np.setdiff1d(np.nonzero(swept[elem_edges].any(axis=1))[0], act)
    els = np.sort(rng.choice(idle, min(500, idle.size), replace=False))
    es = np.unique(elem_edges[els][swept[elem_edges[els]]])
    a, b = edge_nodes[es, 0], edge_nodes[es, 1]
    L, R = edge_elems[es, 0], edge_elems[es, 1]
    hasR = R >= 0
    Rs = np.where(hasR, R, L)
    ers = np.where(hasR, edge_local[es, 1], edge_local[es, 0])
    P = np.stack([np.column_stack([S0["X"][a], S0["nk"][a] * delta]),
                  np.column_stack([S0["X"][b], S0["nk"][b] * delta]),
                  np.column_stack([S1["X"][b], S1["nk"][b] * delta]),
                  np.column_stack([S1["X"][a], S1["nk"][a] * delta])], axis=1)
    ticks = np.stack([S0["nk"][a], S0["nk"][b], S1["nk"][b], S1["nk"][a]], 1).astype(float)
    bc = np.where(hasR, 0, 1)
    G, _ = patch_batch(2, cfg, P, ticks, S0["n"][L], S0["s"][L], S0["trace"][L, edge_local[es, 0]],
                       S0["n"][Rs], S0["s"][Rs], S0["trace"][Rs, ers], hasR, bc, S0["avg"][L])
    dQM = np.zeros((NE, 4))
    np.subtract.at(dQM, L, G)
    np.add.at(dQM, R[hasR], G[hasR])
    got = S1["QM"][els] - S0["QM"][els]
    assert np.abs(got - dQM[els]).max() <= TOL * np.abs(S1["QM"][els]).max()
    assert np.abs(got).max() > 0
    # reconstruction of updated elements from their placed stencils
    samp = np.sort(rng.choice(act, 1000, replace=False))
    sten = stencils_of(mesh.nodes, tris, 2, samp)
    valid = sten[:, :, 0] >= 0
    ss = np.where(sten >= 0, sten, samp[:, None, None])
    fake = SimpleNamespace(cfg=cfg, st=SimpleNamespace(n=S1["n"], s=S1["s"], delta=delta, Xe=S1["Xe"],
                                                       vvel=S1["vvel"], avg=S1["avg"], Q=S1["Q"]))
    Xs, Qs = Solver._virtual(fake, ss, np.broadcast_to(S1["n"][samp][:, None, None], ss.shape))
    wnod_o, _, _, _ = reconstruct_batch(2, cfg, S1["Xe"][samp], S1["Q"][samp], Xs, Qs, valid)
    assert rel(S1["wnod"][samp], wnod_o) < TOL
    # the new predictors of the updated elements that stay short of the macro-step end
    going = samp[S1["n"][samp] < MACRO_TICKS]
    pr = predictor_batch(2, cfg, S1["wnod"][going], S1["Xe"][going], S1["s"][going] * delta,
                         np.zeros(going.size))
    assert rel(S1["trace"][going], pr["trace"]) < TOL
    assert rel(S1["avg"][going], pr["avg"]) < TOL
    assert rel(S1["vvel"][going], pr["vvel"]) < TOL
    print(f"checked {kk.size} nodes, {es.size} patches of {els.size} elements, {samp.size} reconstructions, "
          f"{going.size} predictors", flush=True)
