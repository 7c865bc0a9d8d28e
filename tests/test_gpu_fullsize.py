"""Parity at workload size: the first cycle of the 80k-triangle vortex (M=2,
3 levels) element by element with launches one by one; the explosion with 4
levels at 30k triangles over two macro steps in the launch configuration the
benchmark times (autotuned settings, captured graphs) and with persistent
grids that stride the active list; the explosion at its full 400k triangles
on sampled elements, and the timed configuration bit-identical to launches
one by one there."""
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
    # per CU (the active lists are ~8x one pass), captured graphs, against
    # default settings launched one by one: bit-identical
    del g
    tg = _gpu_solver(mesh, Q0, 2, 4)
    tg.set_tune(sched_chunk=256, list_wg_per_cu=1)
    eg = _gpu_solver(mesh, Q0, 2, 4)
    eg.set_graphs(False)
    st_t, st_e = tg.step_lts(1.0, 2), eg.step_lts(1.0, 2)
    Qt, Xt, tt = tg.download()
    Qe, Xe2, te = eg.download()
    print(f"timed configuration: updates {st_t['element_updates']} / {st_e['element_updates']}", flush=True)
    assert st_t["element_updates"] == st_e["element_updates"] == st["element_updates"]
    assert np.array_equal(Qt, Qe) and np.array_equal(Xt, Xe2) and np.array_equal(tt, te)
    assert np.array_equal(Qe, Q) and np.array_equal(Xe2, X)
