"""Schedule replay (ader_set_schedule_replay): the GPU path takes the steps
that the oracle took, element by element, so that a step decision made in
floating point on both sides (a CFL step at a level boundary, the floor of a
free step) cannot flip between them. Checked with the oracle's own schedule
(no step differs from the kernels' rule) and with a schedule the oracle was
forced into (every replayed change shows up as an override and the results
still agree)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from test_gpu_parity import CASES, TOL, _gpu_solver, _oracle, _span, rel_groups  # noqa: E402

pytestmark = pytest.mark.gpu


def _compare(g, o, mesh):
    Q, X, _ = g.download()
    st = g.stats()
    assert st["element_updates"] == o.st.updates
    assert st["patches"] == o.st.patches and st["node_moves"] == o.st.node_moves
    assert abs(st["t"] - o.st.T) <= 1e-14 * o.st.T
    assert (rel_groups(Q, o.st.Q) < TOL).all()
    assert np.abs(X - o.st.X).max() < TOL * _span(mesh)
    return st


@pytest.mark.parametrize("name,levels,t_end", [("vortex_M2", 0, 0.02), ("explosion_M2", 3, 10.0)])
def test_replay_of_the_oracles_schedule(name, levels, t_end):
    make, M = CASES[name]
    mesh, Q0 = make()
    o = _oracle(mesh, Q0, M, levels)
    if levels:
        o.run(t_end, max_macro_steps=2)
    else:
        o.run(t_end)
    g = _gpu_solver(mesh, Q0, M, levels)
    g.set_schedule_replay(o.step_log)
    g.step_lts(t_end, 2 if levels else 0)
    st = _compare(g, o, mesh)
    print(f"{name}: {sum(len(x) for x in o.step_log)} replayed steps, overrides {st['replay_overrides']}",
          flush=True)
    assert st["replay_overrides"] == 0


def test_replay_of_a_forced_schedule():
    """The oracle halves the first step of every element whose rule allows
    more than the finest nominal step, and of a seeded tenth of the later
    decisions where the step allows it; the GPU replays that schedule."""
    make, M = CASES["explosion_M2"]
    mesh, Q0 = make()
    o = _oracle(mesh, Q0, M, 3)
    rng = np.random.default_rng(17)
    forced = []

    def hook(i, k, p):
        finest = o.st.N >> 2                      # nominal finest step of 3 levels
        if p > finest and (k == 0 or rng.random() < 0.1):
            forced.append((i, k))
            return p // 2
        return p

    o.step_hook = hook
    o.run(10.0, max_macro_steps=2)
    assert len(forced) > 100
    g = _gpu_solver(mesh, Q0, M, 3)
    g.set_schedule_replay(o.step_log)
    g.step_lts(10.0, 2)
    st = _compare(g, o, mesh)
    print(f"forced {len(forced)} steps, overrides {st['replay_overrides']}", flush=True)
    assert st["replay_overrides"] >= len(forced)
    # replay off: the kernels' own rule again, on a fresh state
    g.set_schedule_replay(None)
    g.upload_state(Q0, 0.0)
    g.step_lts(10.0, 2)
    assert g.stats()["replay_overrides"] == 0
    assert g.stats()["element_updates"] != o.st.updates


def test_replay_errors_on_a_short_schedule():
    from paper_1408_3719_amd import AderError
    make, M = CASES["vortex_M2"]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, 3)
    g.set_schedule_replay([[] for _ in range(mesh.n_elems)])
    with pytest.raises(AderError, match="schedule replay"):
        g.step_lts(10.0, 1)
    with pytest.raises(ValueError):
        g.set_schedule_replay([[1]])
