"""Pins of the oracle's reference-element tables against closed forms."""
import math
import os

import numpy as np
import pytest

from oracle import tables as tb

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, *v = line.split()
        out[k] = np.array([float(x) for x in v])
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_legendre_exact_degree(n):
    x, w = tb.gauss_legendre01(n)
    for k in range(2 * n):
        assert abs((w * x ** k).sum() - 1.0 / (k + 1)) < 1e-15
    # one degree beyond the exactness limit must fail (the rule is not over-claimed)
    assert abs((w * x ** (2 * n)).sum() - 1.0 / (2 * n + 1)) > 1e-8


@pytest.mark.parametrize("n", [1, 2, 3, 4, 6])
def test_duffy_rule_monomials(n):
    xi, eta, w = tb.duffy_rule(n)
    for a in range(2 * n - 1):
        for b in range(2 * n - 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs((w * xi ** a * eta ** b).sum() - exact) < 1e-15


@pytest.mark.parametrize("M", [1, 2, 3])
def test_psi_orthonormal_and_constant_first(M):
    xi, eta, w = tb.duffy_rule(M + 2)
    P = tb.eval_psi(M, xi, eta)
    G = np.einsum("pl,pm,p->lm", P, P, w) / w.sum()
    assert np.abs(G - np.eye(P.shape[1])).max() < 1e-13
    assert np.allclose(P[:, 0], 1.0)


def _psi_coeffs_of(M, fn):
    xi, eta, w = tb.duffy_rule(M + 3)
    P = tb.eval_psi(M, xi, eta)
    return np.einsum("pl,p->l", P, fn(xi, eta) * w) / w.sum()


@pytest.mark.parametrize("M,fn,exact", [
    (2, lambda x, y: x * x, 7.0 / 3.0),          # 1/3 (d_xi) + 2 (d_xi^2)
    (2, lambda x, y: x * y, 2.0 / 3.0),          # 1/12 + 1/12 + 1/2
    (3, lambda x, y: x ** 3, 21.3),              # 0.3 + 3 + 18
    (1, lambda x, y: 2 * x - y, 2.5),            # (4 + 1) * 1/2
])
def test_sigma_closed_forms(M, fn, exact):
    """sigma = sum_{1<=a+b<=M} int_Te (d^{ab} p)^2, computed by hand."""
    c = _psi_coeffs_of(M, fn)
    assert abs(c @ tb.sigma_matrix(M) @ c - exact) < 1e-11


@pytest.mark.parametrize("M", [1, 2, 3])
def test_sigma_vanishes_for_constants(M):
    S = tb.sigma_matrix(M)
    assert np.all(S[0] == 0) and np.all(S[:, 0] == 0)


def test_time_matrices_M1_golden():
    g = _golden("time_matrices_M1.txt")
    _, f = tb.time_matrices(1)
    assert np.allclose(f["Kt"].ravel(), g["Kt"], atol=1e-16)
    assert np.allclose(f["Mt"].ravel(), g["Mt"], atol=1e-16)
    assert np.allclose(f["At"].ravel(), g["At"], atol=1e-16)
    assert np.allclose(f["Bt"], g["Bt"], atol=1e-16)


@pytest.mark.parametrize("M", [1, 2, 3])
def test_time_system_exact_for_low_degree_rhs(M):
    """For P of degree <= M-1 the Galerkin solution is the exact integral:
    q(tau_q) = q_0 + dt * int_0^tau_q P, so Bt = 1 and At P = int P."""
    _, f = tb.time_matrices(M)
    tn = tb.time_nodes(M)
    assert np.allclose(f["Bt"], 1.0, atol=1e-14)
    for d in range(M):
        P = tn ** d
        assert np.allclose(f["At"] @ P, tn[1:] ** (d + 1) / (d + 1), atol=1e-14)
    # K11 invertible (the reduced system is well posed)
    e, _ = tb.time_matrices(M)
    K11 = np.array([[float(x) for x in r[1:]] for r in e["Kt"][1:]])
    assert abs(np.linalg.det(K11)) > 1e-3


@pytest.mark.parametrize("M", [1, 2, 3])
def test_nodal_tables_on_polynomials(M):
    rng = np.random.default_rng(M)
    mons = tb.monomials(M)
    c = rng.normal(size=len(mons))

    def p(x, y):
        return sum(ci * x ** a * y ** b for ci, (a, b) in zip(c, mons))

    def px(x, y):
        return sum(ci * a * x ** max(a - 1, 0) * y ** b for ci, (a, b) in zip(c, mons))

    def py(x, y):
        return sum(ci * b * x ** a * y ** max(b - 1, 0) for ci, (a, b) in zip(c, mons))

    nodes = tb.nodal_xy(M)
    vals = p(nodes[:, 0], nodes[:, 1])
    nt = tb.nodal_tables(M)
    assert np.allclose(nt["Dxi"] @ vals, px(nodes[:, 0], nodes[:, 1]), atol=1e-12)
    assert np.allclose(nt["Deta"] @ vals, py(nodes[:, 0], nodes[:, 1]), atol=1e-12)
    mean = 2 * sum(ci * math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
                   for ci, (a, b) in zip(c, mons))
    assert abs(nt["amean"] @ vals - mean) < 1e-12
    chi, _ = tb.gauss_legendre01(M + 1)
    V = [(0, 0), (1, 0), (0, 1)]
    for e in range(3):
        (x0, y0), (x1, y1) = V[e], V[(e + 1) % 3]
        exp = p(x0 + (x1 - x0) * chi, y0 + (y1 - y0) * chi)
        assert np.allclose(nt["edge"][e] @ vals, exp, atol=1e-12)
    vi = tb.vertex_node_index(M)
    assert np.allclose(nodes[vi], np.array(V, float))


@pytest.mark.parametrize("M", [1, 2, 3])
def test_time_integral_and_lagrange(M):
    tn = tb.time_nodes(M)
    L = tb.lagrange_time(M, tn)
    assert np.allclose(L, np.eye(M + 1), atol=1e-15)
    t0, t1 = 0.2, 0.7
    I = tb.lagrange_time_integral(M, np.array(t0), np.array(t1))
    for d in range(M + 1):
        assert abs(I @ tn ** d - (t1 ** (d + 1) - t0 ** (d + 1)) / (d + 1)) < 1e-15
