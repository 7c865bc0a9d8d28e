"""Macro steps replayed from one captured HIP graph against the same kernels
launched one by one: bit-identical states, times and counters, over several
replays with host work (synchronisation, downloads) between them, and after
the target time changes (the graph is captured again)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from test_gpu_parity import CASES, _gpu_solver  # noqa: E402

pytestmark = pytest.mark.gpu

COUNTERS = ("element_updates", "cycles", "macro_steps", "predictor_evals", "patches", "node_moves")


def _same(a, b):
    Qa, Xa, ta = a.download()
    Qb, Xb, tb = b.download()
    return np.array_equal(Qa, Qb) and np.array_equal(Xa, Xb) and np.array_equal(ta, tb)


@pytest.mark.parametrize("name,levels", [("vortex_M2", 3), ("sod_M2", 1), ("explosion_M2", 3),
                                         ("vortex_M3", 2)])
def test_graph_replays_equal_eager_launches(name, levels):
    make, M = CASES[name]
    mesh, Q0 = make()
    print(f"{name} levels={levels} {mesh.n_elems} triangles", flush=True)
    g = _gpu_solver(mesh, Q0, M, levels)          # graphs are the default
    e = _gpu_solver(mesh, Q0, M, levels)
    e.set_graphs(False)
    step = (lambda s, n: s.step_gts(10.0, n)) if levels == 1 else (lambda s, n: s.step_lts(10.0, n))
    for k in range(3):                            # the same graph replayed across calls
        sg, se = step(g, 2), step(e, 2)
        assert _same(g, e), k
        for f in COUNTERS:
            assert sg[f] == se[f], (k, f)
        assert sg["t"] == se["t"]
    # a new target time captures a new graph
    t1 = g.stats()["t"] * 1.2
    sg = g.step_lts(t1, 0) if levels > 1 else g.step_gts(t1, 0)
    se = e.step_lts(t1, 0) if levels > 1 else e.step_gts(t1, 0)
    assert _same(g, e)
    assert sg["t"] == se["t"] and abs(sg["t"] - t1) <= 1e-12 * t1
    for f in COUNTERS:
        assert sg[f] == se[f], f


def test_autotune_keeps_state_and_results():
    """The autotuner restores the state it tuned on, and the tuned launch
    settings give bit-identical results (they only change work grouping)."""
    make, M = CASES["explosion_M2"]
    mesh, Q0 = make()
    a = _gpu_solver(mesh, Q0, M, 3)
    b = _gpu_solver(mesh, Q0, M, 3)
    a.step_lts(10.0, 1)
    b.step_lts(10.0, 1)
    before = a.stats()
    Qa0, Xa0, _ = a.download()
    choice = a.autotune(2)
    print("tuned", choice, flush=True)
    assert choice["ms_per_macro_step"] > 0.0
    after = a.stats()
    Qa1, Xa1, _ = a.download()
    assert np.array_equal(Qa0, Qa1) and np.array_equal(Xa0, Xa1)
    for f in COUNTERS + ("t",):
        assert before[f] == after[f], f
    sa, sb = a.step_lts(10.0, 3), b.step_lts(10.0, 3)
    assert _same(a, b)
    for f in COUNTERS + ("t",):
        assert sa[f] == sb[f], f
    # explicit extreme settings as well
    b.set_tune(sched_chunk=32, list_wg_per_cu=1, sweep_wg_per_cu=1)
    a.set_tune(sched_chunk=1024, list_wg_per_cu=64, sweep_wg_per_cu=64)
    a.step_lts(10.0, 2), b.step_lts(10.0, 2)
    assert _same(a, b)


@pytest.mark.parametrize("name", ["vortex_M2", "explosion_M2"])
def test_free_steps_graph_equals_eager(name):
    """Free local steps: batches of cycles replayed from one captured graph,
    over three successive target times, against launches one by one."""
    make, M = CASES[name]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, 0)
    e = _gpu_solver(mesh, Q0, M, 0)
    e.set_graphs(False)
    for k, t in enumerate((0.004, 0.01, 0.02)):
        sg, se = g.step_lts(t), e.step_lts(t)
        assert _same(g, e), k
        for f in COUNTERS + ("t", "cfl_overshoots"):
            assert sg[f] == se[f], (k, f)
        assert sg["t"] == t and sg["macro_steps"] == k + 1
