"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: relative L-infinity <= 1e-10 per variable group (density; momentum;
total energy), node coordinates within 1e-10 of the domain size, integer
ticks and levels bit-exact.
"""
import numpy as np
import pytest

from oracle.scheme import Config as OConfig
from oracle.scheme import Solver as OSolver
from workloads import explosion_case, sod_case, vortex_case

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _gpu_solver(mesh, Q0, M, levels, mode="lagrangian", flux="rusanov"):
    from paper_1408_3719_amd import Config, Solver
    return Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0,
                  Config(M=M, levels=levels, mesh_velocity=mode, flux=flux))


def _oracle(mesh, Q0, M, levels, mode="lagrangian", flux="rusanov"):
    return OSolver(mesh.nodes, mesh.tris, Q0,
                   OConfig(M=M, levels=levels, mesh_velocity=mode, flux=flux), bedges=mesh.bedges)


def rel_groups(Qg, Qo):
    """Relative L-inf error per group: rho, momentum, total energy."""
    out = []
    for cols in ((0,), (1, 2), (3,)):
        d = np.abs(Qg[:, cols] - Qo[:, cols]).max()
        out.append(d / max(np.abs(Qo[:, cols]).max(), 1e-300))
    return np.array(out)


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _span(mesh):
    return float(np.ptp(mesh.nodes, axis=0).max())


def small_cases():
    return {
        "sod_M1": (lambda: sod_case(600, seed=11), 1),
        "sod_M2": (lambda: sod_case(600, seed=11), 2),
        "vortex_M2": (lambda: vortex_case(900, seed=5), 2),
        "vortex_M3": (lambda: vortex_case(900, seed=5), 3),
        "explosion_M2": (lambda: explosion_case(1500, seed=7), 2),
    }


CASES = small_cases()


@pytest.mark.parametrize("name", list(CASES))
def test_preprocessing_parity(name):
    """First reconstruction and CFL step of every element (paper Sec. 2.6)."""
    make, M = CASES[name]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, 3)
    o = _oracle(mesh, Q0, M, 3)
    wn = g.dump("WNOD")                      # (nb, 4, NE)
    assert rel(np.transpose(wn, (2, 0, 1)), o.st.wnod) < TOL
    assert rel(g.dump("DTCFL"), o.st.dtcfl) < TOL


@pytest.mark.parametrize("name", list(CASES))
def test_macro_begin_parity(name):
    """Levels (bit-exact) and the predictor published for every element."""
    make, M = CASES[name]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, 3)
    o = _oracle(mesh, Q0, M, 3)
    g.debug_macro_begin(10.0, 3)
    o.macro_begin(10.0)
    sc = g.dump("SCAL")
    assert abs(sc[1] - o.st.delta) <= 1e-14 * o.st.delta
    assert np.array_equal(g.dump("STEP"), o.st.s)
    assert rel(np.transpose(g.dump("AVG"), (2, 0, 1)), o.st.avg) < TOL
    assert rel(np.moveaxis(g.dump("TRACE"), -1, 0), o.st.trace) < TOL
    assert rel(np.moveaxis(g.dump("VVEL"), -1, 0), o.st.vvel) < TOL


@pytest.mark.parametrize("name", list(CASES))
def test_single_cycles_parity(name):
    """Cycle by cycle through one macro step of 3 levels: active sets, node
    motion, memory variables, updates, projections, WENO, levels, predictors."""
    make, M = CASES[name]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, 3)
    o = _oracle(mesh, Q0, M, 3)
    g.debug_macro_begin(10.0, 3)
    o.macro_begin(10.0)
    span = _span(mesh)
    for c in range(4):
        o.cycle()
        g.debug_cycles(1)
        assert np.array_equal(g.dump("TICK"), o.st.n), c
        assert np.array_equal(g.dump("STEP"), o.st.s), c
        assert np.array_equal(g.dump("NTICK"), o.st.nk), c
        assert (rel_groups(g.dump("Q").T, o.st.Q) < TOL).all(), c
        assert np.abs(g.dump("X").T - o.st.X).max() < TOL * span, c
        scale = np.abs(o.st.A[:, None] * o.st.Q).max()
        assert np.abs(g.dump("QM").T - o.st.QM).max() < TOL * scale, c
        assert rel(np.transpose(g.dump("WNOD"), (2, 0, 1)), o.st.wnod) < TOL, c
        live = o.st.s > 0
        if live.any():
            tr = np.moveaxis(g.dump("TRACE"), -1, 0)
            assert rel(tr[live], o.st.trace[live]) < TOL, c
            vv = np.moveaxis(g.dump("VVEL"), -1, 0)
            assert rel(vv[live], o.st.vvel[live]) < TOL, c


@pytest.mark.parametrize("name,levels,steps", [
    ("sod_M1", 1, 3), ("sod_M2", 1, 6), ("vortex_M2", 3, 3), ("vortex_M3", 3, 2),
    ("explosion_M2", 3, 3), ("explosion_M2", 1, 4)])
def test_end_to_end_parity(name, levels, steps):
    make, M = CASES[name]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, levels)
    o = _oracle(mesh, Q0, M, levels)
    if levels == 1:
        stg = g.step_gts(10.0, steps)
    else:
        stg = g.step_lts(10.0, steps)
    o.run(10.0, max_macro_steps=steps)
    Q, X, t = g.download()
    assert stg["macro_steps"] == steps
    assert stg["element_updates"] == o.st.updates
    assert stg["node_moves"] == o.st.node_moves and stg["patches"] == o.st.patches
    assert abs(stg["t"] - o.st.T) <= 1e-13 * o.st.T
    assert (rel_groups(Q, o.st.Q) < TOL).all(), rel_groups(Q, o.st.Q)
    assert np.abs(X - o.st.X).max() < TOL * _span(mesh)
    assert np.allclose(t, o.st.T, rtol=1e-13)
    assert stg["max_gcl_residual"] < 1e-13


def test_eulerian_mode_parity():
    mesh, Q0 = vortex_case(900, seed=5)
    g = _gpu_solver(mesh, Q0, 2, 3, mode="eulerian")
    o = _oracle(mesh, Q0, 2, 3, mode="eulerian")
    g.step_lts(10.0, 2)
    o.run(10.0, max_macro_steps=2)
    Q, X, _ = g.download()
    assert (rel_groups(Q, o.st.Q) < TOL).all()
    assert np.array_equal(X, mesh.nodes)


def test_gts_reaches_target_time_exactly():
    mesh, Q0 = sod_case(600, seed=11)
    g = _gpu_solver(mesh, Q0, 2, 1)
    st = g.step_gts(0.01)
    assert abs(st["t"] - 0.01) < 1e-15
    _, _, t = g.download()
    assert np.allclose(t, 0.01, rtol=0, atol=1e-15)


def test_error_on_nonphysical_state():
    from paper_1408_3719_amd import AderError
    mesh, Q0 = sod_case(600, seed=11)
    Q0 = Q0.copy()
    Q0[5, 3] = -1.0
    with pytest.raises(AderError, match="E_STATE"):
        _gpu_solver(mesh, Q0, 1, 1)


@pytest.mark.parametrize("flux", ["osher", "hll"])
@pytest.mark.parametrize("name,levels,steps", [
    ("sod_M2", 1, 4), ("sod_M1", 1, 3), ("explosion_M2", 3, 3), ("vortex_M2", 3, 2)])
def test_flux_end_to_end_parity(flux, name, levels, steps):
    """Osher-type (eq. eqn.osher) and HLL fluxes through the same path."""
    make, M = CASES[name]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, levels, flux=flux)
    o = _oracle(mesh, Q0, M, levels, flux=flux)
    stg = g.step_gts(10.0, steps) if levels == 1 else g.step_lts(10.0, steps)
    o.run(10.0, max_macro_steps=steps)
    Q, X, _ = g.download()
    assert stg["element_updates"] == o.st.updates
    assert (rel_groups(Q, o.st.Q) < TOL).all(), rel_groups(Q, o.st.Q)
    assert np.abs(X - o.st.X).max() < TOL * _span(mesh)
    assert stg["max_gcl_residual"] < 1e-13


def test_osher_single_cycles_parity():
    """Cycle by cycle with the Osher flux: memory variables isolate the patches."""
    make, M = CASES["explosion_M2"]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, 3, flux="osher")
    o = _oracle(mesh, Q0, M, 3, flux="osher")
    g.debug_macro_begin(10.0, 3)
    o.macro_begin(10.0)
    for c in range(4):
        o.cycle()
        g.debug_cycles(1)
        scale = np.abs(o.st.A[:, None] * o.st.Q).max()
        assert np.abs(g.dump("QM").T - o.st.QM).max() < TOL * scale, c
        assert (rel_groups(g.dump("Q").T, o.st.Q) < TOL).all(), c


FREE_CASES = [("sod_M2", 0.01), ("vortex_M2", 0.1), ("vortex_M3", 0.05), ("explosion_M2", 0.01)]


@pytest.mark.parametrize("name,t_end", FREE_CASES)
def test_free_steps_end_to_end_parity(name, t_end):
    """Free local steps (levels = 0): one macro step of 2^30 ticks to t_end,
    every element at floor(dt_CFL / delta) ticks; ticks, update counts and the
    final time exact, states to the parity tolerance."""
    make, M = CASES[name]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, 0)
    o = _oracle(mesh, Q0, M, 0)
    stg = g.step_lts(t_end)
    o.run(t_end)
    Q, X, t = g.download()
    print(f"{name} updates {stg['element_updates']} oracle cycles {o.st.cycles} "
          f"launched {stg['cycles']}", flush=True)
    assert stg["macro_steps"] == o.st.macro_steps == 1
    assert stg["element_updates"] == o.st.updates
    assert stg["node_moves"] == o.st.node_moves and stg["patches"] == o.st.patches
    assert stg["cfl_overshoots"] == o.st.cfl_overshoots == 0
    assert stg["cycles"] == 16 * -(-o.st.cycles // 16)      # launched in batches of 16
    assert stg["t"] == o.st.T == t_end
    assert (rel_groups(Q, o.st.Q) < TOL).all(), rel_groups(Q, o.st.Q)
    assert np.abs(X - o.st.X).max() < TOL * _span(mesh)
    assert (t == t_end).all()
    assert stg["max_gcl_residual"] < 1e-13


@pytest.mark.parametrize("name,t_end", [("vortex_M2", 0.1), ("explosion_M2", 0.01)])
def test_free_steps_single_cycles_parity(name, t_end):
    """Cycle by cycle through a free-step interval: ticks and steps (not powers
    of two, no alignment) bit-exact, states and node motion to tolerance."""
    make, M = CASES[name]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, 0)
    o = _oracle(mesh, Q0, M, 0)
    g.debug_macro_begin(t_end, 0)
    o.macro_begin(t_end)
    assert g.dump("SCAL")[1] == o.st.delta
    assert np.array_equal(g.dump("STEP"), o.st.s)
    assert (o.st.s & (o.st.s - 1) != 0).any()               # genuinely free steps
    span = _span(mesh)
    for c in range(6):
        o.cycle()
        g.debug_cycles(1)
        assert np.array_equal(g.dump("TICK"), o.st.n), c
        assert np.array_equal(g.dump("STEP"), o.st.s), c
        assert np.array_equal(g.dump("NTICK"), o.st.nk), c
        assert (rel_groups(g.dump("Q").T, o.st.Q) < TOL).all(), c
        assert np.abs(g.dump("X").T - o.st.X).max() < TOL * span, c
        live = o.st.s > 0
        tr = np.moveaxis(g.dump("TRACE"), -1, 0)
        assert rel(tr[live], o.st.trace[live]) < TOL, c


@pytest.mark.parametrize("levels", [1, 3, 0])
def test_target_time_already_reached_is_a_no_op(levels):
    """A target at or before the current time takes no step and leaves the
    state bit for bit; stepping on afterwards works as from a fresh start."""
    make, M = CASES["vortex_M2"]
    mesh, Q0 = make()
    g = _gpu_solver(mesh, Q0, M, levels)
    step = g.step_gts if levels == 1 else g.step_lts
    first = step(0.02)
    Qa, Xa, ta = g.download()
    for t in (0.02, 0.01, 0.0, -1.0):
        st = step(t)
        Qb, Xb, tb = g.download()
        assert np.array_equal(Qa, Qb) and np.array_equal(Xa, Xb) and np.array_equal(ta, tb), t
        for f in ("element_updates", "cycles", "macro_steps"):
            assert st[f] == first[f], (t, f)
    st = step(0.03)
    assert abs(st["t"] - 0.03) <= 1e-13 and st["element_updates"] > first["element_updates"]
