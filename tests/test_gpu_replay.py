"""Schedule replay (ader_set_schedule_replay): the GPU path takes the steps
that the oracle took, element by element, so that a step decision made in
floating point on both sides (a CFL step at a level boundary, the floor of a
free step) cannot flip between them. Checked with the oracle's own schedule
(no step differs from the kernels' rule) and with a schedule the oracle was
forced into (every replayed change shows up as an override and the results
still agree). The schedule record (ader_set_schedule_record) gives back a
replayed schedule exactly, and a recorded run with its tick lengths
(ader_set_delta_replay) replays bit for bit."""
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


def test_record_of_a_replayed_oracle_schedule():
    """Recording while replaying the oracle's schedule gives back the oracle's
    steps exactly and its tick lengths to rounding."""
    from oracle.adjoint import lts_schedule
    make, M = CASES["explosion_M2"]
    mesh, Q0 = make()
    o = _oracle(mesh, Q0, M, 3)
    sched = lts_schedule(o, 10.0, 2)
    g = _gpu_solver(mesh, Q0, M, 3)
    g.set_schedule_replay(o.step_log)
    g.record_schedule(64, 4)
    g.step_lts(10.0, 2)
    log, deltas = g.recorded_schedule()
    assert log == [list(x) for x in o.step_log]
    assert len(deltas) == 2
    for d, (od, _) in zip(deltas, sched):
        assert abs(d - od) <= 1e-14 * od


def test_recorded_schedule_replays_bit_for_bit():
    """A run's recorded steps and tick lengths, replayed from the same data,
    give the same run bit for bit with no step overridden; from perturbed data
    the replayed schedule is the one taken (the record of the second run equals
    the first's), and running past the recorded tick lengths is refused."""
    from paper_1408_3719_amd import AderError
    make, M = CASES["explosion_M2"]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, 3)
    g.record_schedule(64, 4)
    g.step_lts(10.0, 3)
    log, deltas = g.recorded_schedule()
    QA, XA, _ = g.download()
    assert len(deltas) == 3 and sum(len(x) for x in log) > 3 * mesh.n_elems
    g.set_schedule_replay(log)
    g.set_delta_replay(deltas)
    g.upload_state(Q0, 0.0)
    g.record_schedule(64, 4)
    g.step_lts(10.0, 3)
    QB, XB, _ = g.download()
    assert np.array_equal(QA, QB) and np.array_equal(XA, XB)
    assert g.stats()["replay_overrides"] == 0
    Qp = Q0 * (1.0 + 1e-4 * np.random.default_rng(9).standard_normal(Q0.shape))
    g.set_schedule_replay(log)
    g.upload_state(Qp, 0.0)
    g.record_schedule(64, 4)
    g.step_lts(10.0, 3)
    log2, deltas2 = g.recorded_schedule()
    assert log2 == log and deltas2 == deltas
    g.set_schedule_replay(log)
    g.upload_state(Q0, 0.0)
    g.record_schedule(0, 0)
    with pytest.raises(AderError, match="tick lengths"):
        g.step_lts(10.0, 4)
