"""Pins of the oracle's Osher-type (eq. eqn.osher, path eq. eqn.path) and HLL
ALE fluxes: finite-difference Jacobian, the matrix absolute value, upwinding,
consistency, symmetry, and the Sod problem against the exact solution."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
from exact_riemann import sample  # noqa: E402

from oracle import euler  # noqa: E402
from oracle.scheme import (Config, Solver, _ale_flux_dot, abs_matrix, ale_jacobian,  # noqa: E402
                           ale_wave_speeds, hll_flux, osher_flux, rusanov_flux)
from workloads import cell_average, sod_primitive, strip_mesh  # noqa: E402

G = 1.4


def _states(rng, n):
    rho = rng.uniform(0.2, 2.0, n)
    u = rng.uniform(-1.5, 1.5, n)
    v = rng.uniform(-1.5, 1.5, n)
    p = rng.uniform(0.1, 3.0, n)
    return np.stack([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v)], -1)


def test_jacobian_is_the_derivative_of_the_ale_flux():
    rng = np.random.default_rng(1)
    q = _states(rng, 20)
    N = rng.normal(size=(20, 3))
    A = ale_jacobian(q, N, G)
    h = 1e-6
    for k in range(4):
        e = np.zeros(4)
        e[k] = h * np.abs(q).max(axis=1).max()
        fd = (_ale_flux_dot(q + e, N, G) - _ale_flux_dot(q - e, N, G)) / (2 * e[k])
        assert np.abs(A[..., :, k] - fd).max() < 1e-7 * np.abs(A).max()


def test_jacobian_eigenvalues_are_the_ale_wave_speeds():
    """u.N_xy + N_t -/+ c |N_xy| and u.N_xy + N_t (twice), against LAPACK."""
    rng = np.random.default_rng(2)
    q = _states(rng, 10)
    N = rng.normal(size=(10, 3))
    lam = ale_wave_speeds(q, N, G)
    want = np.sort(np.concatenate([lam, lam[:, 1:2]], -1), axis=-1)
    got = np.sort(np.linalg.eigvals(ale_jacobian(q, N, G)).real, axis=-1)
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


def test_abs_matrix():
    """|A| against R |Lambda| R^-1 from LAPACK on well-separated cases; |A|^2 = A^2;
    |A| = A (= -A) when every wave speed is positive (negative)."""
    rng = np.random.default_rng(3)
    q = _states(rng, 10)
    N = rng.normal(size=(10, 3))
    A = ale_jacobian(q, N, G)
    B = abs_matrix(A, ale_wave_speeds(q, N, G))
    lam, R = np.linalg.eig(A)
    ref = (R @ (np.abs(lam.real)[..., :, None] * np.linalg.inv(R))).real
    assert np.abs(B - ref).max() < 1e-10 * np.abs(ref).max()
    assert np.abs(B @ B - A @ A).max() < 1e-11 * np.abs(A @ A).max()
    Np = N.copy()
    Np[:, 2] = 20.0 * (1 + np.abs(N).sum(axis=1))          # mesh sweeping fast: all speeds > 0
    Ap = ale_jacobian(q, Np, G)
    assert np.abs(abs_matrix(Ap, ale_wave_speeds(q, Np, G)) - Ap).max() < 1e-12 * np.abs(Ap).max()
    An = ale_jacobian(q, -Np, G)
    assert np.abs(abs_matrix(An, ale_wave_speeds(q, -Np, G)) + An).max() < 1e-12 * np.abs(An).max()
    # a gas at rest through a static face: |A| has the acoustic part only
    q0 = np.array([[1.0, 0.0, 0.0, 2.5]])
    N0 = np.array([[1.0, 0.0, 0.0]])
    A0 = ale_jacobian(q0, N0, G)
    B0 = abs_matrix(A0, ale_wave_speeds(q0, N0, G))
    assert np.abs(B0 @ B0 - A0 @ A0).max() < 1e-13


@pytest.mark.parametrize("flux", [osher_flux, hll_flux, rusanov_flux])
def test_consistency_and_symmetry(flux):
    """F(q, q, N) = F~(q).N, and F(qr, ql, -N) = -F(ql, qr, N)."""
    rng = np.random.default_rng(4)
    ql, qr = _states(rng, 16), _states(rng, 16)
    N = rng.normal(size=(16, 3))
    f = flux(ql, ql, N, G)
    assert np.abs(f - _ale_flux_dot(ql, N, G)).max() < 1e-14 * np.abs(f).max()
    a, b = flux(ql, qr, N, G), flux(qr, ql, -N, G)
    assert np.abs(a + b).max() < 1e-13 * np.abs(a).max()


def test_osher_upwinds_when_all_waves_move_one_way():
    """With every wave speed positive along the whole path, |A| = A and the path
    integral of A dq is F(qr) - F(ql): the Osher flux is F~(ql).N, exactly in the
    limit of many Gauss points and to quadrature accuracy with three."""
    rng = np.random.default_rng(5)
    ql = _states(rng, 8)
    qr = ql * (1 + 0.05 * rng.normal(size=ql.shape))
    N = rng.normal(size=(8, 3))
    N[:, 2] = 20.0 * (1 + np.abs(N).sum(axis=1))
    fl = _ale_flux_dot(ql, N, G)
    many = osher_flux(ql, qr, N, G, npts=24)
    assert np.abs(many - fl).max() < 1e-11 * np.abs(fl).max()
    three = osher_flux(ql, qr, N, G)
    assert np.abs(three - fl).max() < 1e-5 * np.abs(fl).max()
    # and the downwind state when every speed is negative
    fr = _ale_flux_dot(qr, -N, G)
    assert np.abs(osher_flux(ql, qr, -N, G, npts=24) - fr).max() < 1e-11 * np.abs(fr).max()


def test_hll_upwinds_exactly():
    rng = np.random.default_rng(6)
    ql, qr = _states(rng, 8), _states(rng, 8)
    N = rng.normal(size=(8, 3))
    N[:, 2] = 50.0 * (1 + np.abs(N).sum(axis=1))
    assert np.array_equal(hll_flux(ql, qr, N, G), _ale_flux_dot(ql, N, G))
    assert np.array_equal(hll_flux(ql, qr, -N, G), _ale_flux_dot(qr, -N, G))


def test_osher_less_dissipative_than_rusanov_on_sod():
    """RP1 (paper Sec. 3.2): with the same mesh, order and time, the Osher-type
    flux gives a smaller L1 density error than the Rusanov flux (the paper's
    motivation for it), and so does HLL."""
    mesh = strip_mesh(-0.5, 0.5, 0.0, 0.1, 0.02, seed=1408, slip_y=True)
    Q0 = cell_average(mesh, sod_primitive, G)
    err = {}
    for f in ("rusanov", "osher", "hll"):
        s = Solver(mesh.nodes, mesh.tris, Q0, Config(M=2, levels=1, flux=f), bedges=mesh.bedges)
        s.run(0.04)
        xc = s.st.Xe.mean(axis=1)[:, 0]
        ex = sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), xc / 0.04)
        err[f] = float((np.abs(s.st.Q[:, 0] - ex[:, 0]) * s.st.A).sum() / s.st.A.sum())
        assert s.st.max_gcl < 1e-13
    assert err["osher"] < err["rusanov"], err
    assert err["hll"] < err["rusanov"], err
