"""RP1, the Sod shock tube (paper Sec. 3.2), on the GPU path to the paper's
final time t = 0.2: the shock-tube workload's 2k-triangle strip (slip walls
at y = 0 and 0.1, transmissive ends), M = 2, global time stepping. The
density approaches the exact Riemann solution, the star-region velocity
plateau sits at the exact star velocity, the wall nodes stay on the walls and
mass changes only by what crosses the open ends (nothing, before the waves
reach them)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from exact_riemann import sample, star_state  # noqa: E402

from workloads import sod_case  # noqa: E402

pytestmark = pytest.mark.gpu

LEFT, RIGHT = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)


def test_sod_to_final_time_against_exact_solution():
    from paper_1408_3719_amd import Config, Solver
    mesh, Q0 = sod_case(2000)
    s = Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=2, levels=1))
    st = s.step_gts(0.2, 100_000)
    assert st["t"] == 0.2 and st["max_gcl_residual"] < 1e-12
    Q, X, _ = s.download()
    p = X[mesh.tris]
    A = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
               - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    xc = p.mean(axis=1)[:, 0] / 0.2
    ex = sample(LEFT, RIGHT, xc)
    l1 = float((A * np.abs(Q[:, 0] - ex[:, 0])).sum() / A.sum())
    print(f"Sod M=2 {mesh.n_elems} triangles, t = 0.2: L1(rho) = {l1:.3e}, "
          f"{st['macro_steps']} steps", flush=True)
    assert l1 < 1e-2
    _, ustar, _, _ = star_state(LEFT, RIGHT)
    u = Q[:, 1] / Q[:, 0]
    plateau = (xc > 0.3) & (xc < 0.8)
    assert abs(np.median(u[plateau]) - ustar) < 0.02
    assert np.abs(X[:, 1] - np.clip(X[:, 1], 0.0, 0.1)).max() == 0.0     # nodes inside the strip
    on_wall = (np.abs(mesh.nodes[:, 1]) < 1e-14) | (np.abs(mesh.nodes[:, 1] - 0.1) < 1e-14)
    assert np.abs(X[on_wall, 1] - mesh.nodes[on_wall, 1]).max() < 1e-12
    mass0 = _areas(mesh.nodes, mesh.tris) @ Q0[:, 0]
    assert abs(A @ Q[:, 0] - mass0) < 1e-12 * mass0


def _areas(nodes, tris):
    p = nodes[tris]
    return 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                  - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
