"""Batched independent simulations (disjoint meshes concatenated, each with
its own time and tick length) through one set of kernel launches: every
instance matches the oracle run of that instance alone, and the GPU run of
that instance alone bit for bit. The target time is reached after different
numbers of macro steps by different instances, so finished instances sit
frozen while the others go on."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from test_gpu_parity import TOL, rel_groups  # noqa: E402

from oracle.scheme import Config as OConfig  # noqa: E402
from oracle.scheme import Solver as OSolver  # noqa: E402
from workloads import batched_cases, concat_instances, explosion_case, sod_case, vortex_case  # noqa: E402

pytestmark = pytest.mark.gpu


def _cases():
    """Six uneven instances (350-900 triangles) that stay physical over the
    tested horizons: shock tube, explosion, vortex and three random Riemann /
    explosion instances of the batched recipe."""
    cases = [sod_case(600, seed=11), explosion_case(900, seed=22), vortex_case(700, seed=23)]
    b = batched_cases(n_instances=8, seed=5, n_min=300, n_max=1200)
    cases += [b[0], b[3], b[7]]
    return cases


@pytest.mark.parametrize("levels,t_target,max_steps", [(3, 10.0, 3), (3, 0.02, 0), (1, 0.003, 0),
                                                      (0, 0.02, 0)])
def test_batch_matches_each_instance_alone(levels, t_target, max_steps):
    from paper_1408_3719_amd import Config, Solver
    cases = _cases()
    nodes, tris, bedges, Q0, first = concat_instances(cases)
    print(f"batch of {len(cases)} instances, {tris.shape[0]} triangles, L={levels}", flush=True)
    cfg = Config(M=2, levels=levels)
    g = Solver(nodes, tris, bedges, Q0, cfg, instance_first=first)
    st = g.step_lts(t_target, max_steps) if levels != 1 else g.step_gts(t_target, max_steps)
    Q, X, t = g.download()
    T = g.instance_times()
    node_off = np.cumsum([0] + [m.nodes.shape[0] for m, _ in cases])
    updates = 0
    for k, (mesh, q0) in enumerate(cases):
        e0, e1 = first[k], first[k + 1]
        v0, v1 = node_off[k], node_off[k + 1]
        o = OSolver(mesh.nodes, mesh.tris, q0, OConfig(M=2, levels=levels), bedges=mesh.bedges)
        o.run(t_target, max_macro_steps=max_steps or None)
        updates += o.st.updates
        assert abs(T[k] - o.st.T) <= 1e-13 * max(1.0, o.st.T), k
        assert (rel_groups(Q[e0:e1], o.st.Q) < TOL).all(), (k, rel_groups(Q[e0:e1], o.st.Q))
        span = float(np.ptp(mesh.nodes, axis=0).max())
        assert np.abs(X[v0:v1] - o.st.X).max() < TOL * span, k
        assert np.allclose(t[e0:e1], o.st.T, rtol=1e-13)
        # the same instance alone on the GPU: identical bits
        a = Solver(mesh.nodes, mesh.tris, mesh.bedges, q0, cfg)
        sa = a.step_lts(t_target, max_steps) if levels != 1 else a.step_gts(t_target, max_steps)
        Qa, Xa, _ = a.download()
        assert np.array_equal(Qa, Q[e0:e1]) and np.array_equal(Xa, X[v0:v1]), k
        assert sa["t"] == T[k]
    assert st["element_updates"] == updates
    if max_steps == 0:
        assert np.allclose(T, t_target, rtol=0, atol=1e-12)
        assert st["t"] == T.min()
