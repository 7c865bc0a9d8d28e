"""Parity at full workload size, in the launch configuration the benchmark
times (80k-triangle vortex mesh, M=2, 3 levels), every element compared; and
the explosion workload with 4 levels at moderate size."""
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


def test_explosion_four_levels_parity():
    mesh, Q0 = explosion_case(12_000, seed=7)
    g = _gpu_solver(mesh, Q0, 2, 4)
    o = _oracle(mesh, Q0, 2, 4)
    st = g.step_lts(1.0, 2)
    o.run(1.0, max_macro_steps=2)
    Q, X, _ = g.download()
    assert st["element_updates"] == o.st.updates
    assert (rel_groups(Q, o.st.Q) < TOL).all()
    assert np.abs(X - o.st.X).max() < TOL * _span(mesh)
    assert o.st.updates < 2 * 8 * mesh.n_elems         # fewer updates than GTS at the finest step
