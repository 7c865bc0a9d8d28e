"""Universal reference-element tables of the scheme (oracle, test infrastructure).

Everything here is defined on the reference triangle T_e = {(0,0),(1,0),(0,1)}
(eq. xietaTransf) and the reference time interval [0,1] (eq. timeTransf):

  * Gauss-Legendre rules on [0,1] (Newton iteration on the Legendre polynomial)
    and the collapsed (Duffy) product rule on T_e;
  * the orthogonal modal basis psi_l of the reconstruction (Sec. 2.2, after
    eq. intConsRec), built here by exact rational Gram-Schmidt on monomials with
    psi_1 = 1, and the oscillation-indicator matrix Sigma (eq. Sigma, summed
    over derivative orders 1 <= alpha+beta <= M);
  * the nodal space-time basis theta = phi_m(xi,eta) * l_q(tau) of the
    predictor (eq. thetaSol) on the equispaced lattice (a/M, b/M) x {q/M};
  * the time parts of the universal matrices K_tau and M of eq. Ktau, and the
    reduced per-node time system obtained when only test functions with
    tau_k > 0 are kept (eq. CGfinal with the tau=0 degrees of freedom fixed).

All rational quantities are exact (fractions.Fraction); floats are produced at
the end.  Not shared with the HIP library, which builds its own tables.
"""
from __future__ import annotations

import functools
import math
from fractions import Fraction

import numpy as np

F = Fraction


# ---------------------------------------------------------------------------
# Quadrature
# ---------------------------------------------------------------------------
def _legendre(n: int, x: float):
    """(P_n(x), P_n'(x)) by the three-term recurrence."""
    p0, p1 = 1.0, x
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    return p1, n * (x * p1 - p0) / (x * x - 1.0)


@functools.lru_cache(maxsize=None)
def gauss_legendre01(n: int):
    """n-point Gauss-Legendre rule on [0,1]: nodes ascending, weights sum to 1.
    Roots of P_n by Newton's method from the usual cosine guesses."""
    xs, ws = [], []
    for i in range(1, n + 1):
        x = math.cos(math.pi * (i - 0.25) / (n + 0.5))
        for _ in range(100):
            p, dp = _legendre(n, x)
            dx = p / dp
            x -= dx
            if abs(dx) < 1e-16:
                break
        _, dp = _legendre(n, x)
        xs.append(x)
        ws.append(2.0 / ((1.0 - x * x) * dp * dp))
    xs = np.array(xs)[::-1]
    ws = np.array(ws)[::-1]
    return 0.5 * (xs + 1.0), 0.5 * ws


@functools.lru_cache(maxsize=None)
def duffy_rule(n: int):
    """Collapsed n x n Gauss rule on T_e: xi = u(1-v), eta = v, Jacobian (1-v).
    Exact for polynomials of total degree <= 2n-2.  Weights sum to |T_e| = 1/2."""
    u, wu = gauss_legendre01(n)
    xi, eta, w = [], [], []
    for i in range(n):
        for j in range(n):
            xi.append(u[i] * (1.0 - u[j]))
            eta.append(u[j])
            w.append(wu[i] * wu[j] * (1.0 - u[j]))
    return np.array(xi), np.array(eta), np.array(w)


# ---------------------------------------------------------------------------
# Exact polynomials in (xi, eta): dict {(a, b): Fraction}
# ---------------------------------------------------------------------------
def monomials(M: int):
    """Exponents (a, b) of the monomials xi^a eta^b, a+b <= M, by total degree."""
    return [(d - b, b) for d in range(M + 1) for b in range(d + 1)]


def int_Te(a: int, b: int) -> Fraction:
    """Exact integral of xi^a eta^b over T_e: a! b! / (a+b+2)!."""
    return F(math.factorial(a) * math.factorial(b), math.factorial(a + b + 2))


def p_mul(p, q):
    out = {}
    for (a1, b1), c1 in p.items():
        for (a2, b2), c2 in q.items():
            k = (a1 + a2, b1 + b2)
            out[k] = out.get(k, F(0)) + c1 * c2
    return out


def p_add(p, q, s=F(1)):
    out = dict(p)
    for k, c in q.items():
        out[k] = out.get(k, F(0)) + s * c
    return out


def p_int(p) -> Fraction:
    return sum((c * int_Te(a, b) for (a, b), c in p.items()), F(0))


def p_diff(p, da: int, db: int):
    out = {}
    for (a, b), c in p.items():
        if a < da or b < db:
            continue
        f = F(math.perm(a, da) * math.perm(b, db))
        out[(a - da, b - db)] = out.get((a - da, b - db), F(0)) + c * f
    return out


def p_coeffs(p, M: int):
    mons = monomials(M)
    return [p.get(m, F(0)) for m in mons]


# ---------------------------------------------------------------------------
# Modal reconstruction basis and Sigma
# ---------------------------------------------------------------------------
@functools.lru_cache(maxsize=None)
def _orthogonal_exact(M: int):
    """Gram-Schmidt of the monomials w.r.t. the mean inner product on T_e
    (<f,g> = 2 * int_Te f g).  Returns the orthogonal polynomials (exact) and
    their squared norms (exact)."""
    polys, norms = [], []
    for m in monomials(M):
        p = {m: F(1)}
        for q, nq in zip(polys, norms):
            proj = 2 * p_int(p_mul({m: F(1)}, q)) / nq
            p = p_add(p, q, -proj)
        polys.append(p)
        norms.append(2 * p_int(p_mul(p, p)))
    return polys, norms


@functools.lru_cache(maxsize=None)
def psi_coeffs(M: int) -> np.ndarray:
    """C (nb x nb): psi_l(xi,eta) = sum_k C[l,k] xi^a_k eta^b_k, orthonormal
    for the mean inner product, psi_1 = 1 (so every psi_l, l>1, has zero mean)."""
    polys, norms = _orthogonal_exact(M)
    C = np.array([[float(c) for c in p_coeffs(p, M)] for p in polys])
    scale = np.array([1.0 / math.sqrt(float(n)) for n in norms])
    return C * scale[:, None]


@functools.lru_cache(maxsize=None)
def sigma_matrix(M: int) -> np.ndarray:
    """Sigma_lm = sum_{1<=alpha+beta<=M} int_Te d^{ab}psi_l d^{ab}psi_m (eq. Sigma;
    the zeroth derivative is excluded so that sigma vanishes for constants)."""
    polys, norms = _orthogonal_exact(M)
    nb = len(polys)
    S = np.zeros((nb, nb))
    for l in range(nb):
        for m in range(nb):
            acc = F(0)
            for order in range(1, M + 1):
                for beta in range(order + 1):
                    alpha = order - beta
                    acc += p_int(p_mul(p_diff(polys[l], alpha, beta), p_diff(polys[m], alpha, beta)))
            S[l, m] = float(acc) / math.sqrt(float(norms[l]) * float(norms[m]))
    return S


def eval_monomials(M: int, xi, eta) -> np.ndarray:
    """Monomial values, shape (..., nb)."""
    xi = np.asarray(xi, float)
    eta = np.asarray(eta, float)
    return np.stack([xi ** a * eta ** b for (a, b) in monomials(M)], axis=-1)


def eval_psi(M: int, xi, eta) -> np.ndarray:
    """psi_l(xi, eta), shape (..., nb)."""
    return eval_monomials(M, xi, eta) @ psi_coeffs(M).T


# ---------------------------------------------------------------------------
# Nodal space-time basis
# ---------------------------------------------------------------------------
@functools.lru_cache(maxsize=None)
def spatial_nodes(M: int):
    """Equispaced lattice (i/M, j/M), i+j <= M, ordered by j then i (exact)."""
    return [(F(i, M), F(j, M)) for j in range(M + 1) for i in range(M + 1 - j)]


def vertex_node_index(M: int):
    """Lattice index of the reference vertices (0,0), (1,0), (0,1)."""
    nodes = spatial_nodes(M)
    return [nodes.index((F(0), F(0))), nodes.index((F(1), F(0))), nodes.index((F(0), F(1)))]


def _solve_exact(A, B):
    """Gauss-Jordan solve A X = B in exact rationals."""
    n = len(A)
    m = len(B[0])
    aug = [list(A[i]) + list(B[i]) for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if aug[r][c] != 0)
        aug[c], aug[piv] = aug[piv], aug[c]
        pv = aug[c][c]
        aug[c] = [x / pv for x in aug[c]]
        for r in range(n):
            if r != c and aug[r][c] != 0:
                f = aug[r][c]
                aug[r] = [x - f * y for x, y in zip(aug[r], aug[c])]
    return [row[n:n + m] for row in aug]


@functools.lru_cache(maxsize=None)
def _phi_exact(M: int):
    """Lagrange basis phi_m on the lattice as exact monomial coefficients:
    phi[m] is the coefficient list, phi_m(node_k) = delta_mk."""
    nodes = spatial_nodes(M)
    mons = monomials(M)
    V = [[x ** a * y ** b for (a, b) in mons] for (x, y) in nodes]      # V[node][mono]
    nb = len(nodes)
    ident = [[F(int(i == j)) for j in range(nb)] for i in range(nb)]
    # coefficients c (mono x basis) with V c = I
    Cm = _solve_exact(V, ident)
    return [{mons[k]: Cm[k][m] for k in range(nb) if Cm[k][m] != 0} for m in range(nb)]


def _p_eval(p, x, y):
    return sum(c * x ** a * y ** b for (a, b), c in p.items())


@functools.lru_cache(maxsize=None)
def nodal_tables(M: int):
    """Dict of float tables of the spatial nodal basis:
      Dxi, Deta (nb x nb): derivative of the interpolant at node m' from nodal values;
      amean (nb): mean over T_e of phi_m (sums to 1);
      edge (3, nG, nb): phi_m at the Gauss points of reference edge e, where edge e
             runs from vertex e to vertex e+1 (mod 3), nG = M+1 points;
      phi_at(xi, eta) evaluator is eval_phi()."""
    phi = _phi_exact(M)
    nodes = spatial_nodes(M)
    nb = len(nodes)
    Dxi = np.array([[float(_p_eval(p_diff(phi[m], 1, 0), *nodes[k])) for m in range(nb)] for k in range(nb)])
    Deta = np.array([[float(_p_eval(p_diff(phi[m], 0, 1), *nodes[k])) for m in range(nb)] for k in range(nb)])
    amean = np.array([float(2 * p_int(phi[m])) for m in range(nb)])
    chi, _ = gauss_legendre01(M + 1)
    verts = [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0)]
    edge = np.zeros((3, M + 1, nb))
    for e in range(3):
        (x0, y0), (x1, y1) = verts[e], verts[(e + 1) % 3]
        for g, c in enumerate(chi):
            edge[e, g] = eval_phi(M, x0 + (x1 - x0) * c, y0 + (y1 - y0) * c)
    return dict(Dxi=Dxi, Deta=Deta, amean=amean, edge=edge)


def eval_phi(M: int, xi, eta) -> np.ndarray:
    """phi_m(xi, eta), shape (..., nb)."""
    phi = _phi_exact(M)
    mons = monomials(M)
    C = np.array([[float(p.get(mn, F(0))) for mn in mons] for p in phi])
    return eval_monomials(M, xi, eta) @ C.T


def nodal_xy(M: int) -> np.ndarray:
    return np.array([[float(x), float(y)] for (x, y) in spatial_nodes(M)])


# ---------------------------------------------------------------------------
# Time basis and the reduced predictor time system
# ---------------------------------------------------------------------------
def time_nodes(M: int) -> np.ndarray:
    return np.array([q / M for q in range(M + 1)])


def lagrange_time(M: int, tau) -> np.ndarray:
    """l_q(tau) = prod_{r != q} (tau - tau_r)/(tau_q - tau_r), shape (..., M+1)."""
    tau = np.asarray(tau, float)
    tn = time_nodes(M)
    out = []
    for q in range(M + 1):
        v = np.ones_like(tau)
        for r in range(M + 1):
            if r != q:
                v = v * (tau - tn[r]) / (tn[q] - tn[r])
        out.append(v)
    return np.stack(out, axis=-1)


def lagrange_time_integral(M: int, t0, t1) -> np.ndarray:
    """int_{t0}^{t1} l_q(tau) dtau by an (M+1)-point Gauss rule (exact), (..., M+1)."""
    t0 = np.asarray(t0, float)
    t1 = np.asarray(t1, float)
    x, w = gauss_legendre01(M + 1)
    acc = 0.0
    for xg, wg in zip(x, w):
        acc = acc + wg * lagrange_time(M, t0 + (t1 - t0) * xg)
    return acc * (t1 - t0)[..., None]


@functools.lru_cache(maxsize=None)
def _time_exact(M: int):
    """Exact univariate Lagrange polynomials l_q as coefficient lists (ascending)."""
    tn = [F(q, M) for q in range(M + 1)]
    polys = []
    for q in range(M + 1):
        c = [F(1)]
        for r in range(M + 1):
            if r == q:
                continue
            den = tn[q] - tn[r]
            # multiply by (tau - tn[r]) / den
            nc = [F(0)] * (len(c) + 1)
            for i, ci in enumerate(c):
                nc[i + 1] += ci / den
                nc[i] -= ci * tn[r] / den
            c = nc
        polys.append(c)
    return polys


def _u_int01(c):
    return sum((ci / (i + 1) for i, ci in enumerate(c)), F(0))


def _u_mul(a, b):
    out = [F(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _u_diff(c):
    return [c[i] * i for i in range(1, len(c))] or [F(0)]


@functools.lru_cache(maxsize=None)
def time_matrices(M: int):
    """Kt[k,l] = int_0^1 l_k l_l' dtau and Mt[k,l] = int_0^1 l_k l_l dtau (time
    factors of K_tau and M, eq. Ktau), and the reduced system
        q_{1:} = Bt q_0 + dt * At P        (rows k = 1..M only; the spatial
    mass matrix cancels because theta is a tensor product), with
        At = Kt[1:,1:]^-1 Mt[1:,:],  Bt = -Kt[1:,1:]^-1 Kt[1:,0].
    Also Dt[q',q] = l_q'(tau_q') for the time derivative at the nodes.
    Returns exact Fractions (lists) and floats (arrays)."""
    L = _time_exact(M)
    n = M + 1
    Kt = [[_u_int01(_u_mul(L[k], _u_diff(L[l]))) for l in range(n)] for k in range(n)]
    Mt = [[_u_int01(_u_mul(L[k], L[l])) for l in range(n)] for k in range(n)]
    K11 = [row[1:] for row in Kt[1:]]
    rhsA = [row[:] for row in Mt[1:]]
    rhsB = [[-Kt[k][0]] for k in range(1, n)]
    At = _solve_exact(K11, rhsA)
    Bt = [r[0] for r in _solve_exact(K11, rhsB)]
    tn = [F(q, M) for q in range(n)]
    Dt = [[sum((c * i * tn[qp] ** (i - 1) for i, c in enumerate(L[q]) if i > 0), F(0))
           for q in range(n)] for qp in range(n)]
    exact = dict(Kt=Kt, Mt=Mt, At=At, Bt=Bt, Dt=Dt)
    fl = {k: np.array([[float(x) for x in row] for row in v]) if isinstance(v[0], list)
          else np.array([float(x) for x in v]) for k, v in exact.items()}
    return exact, fl


# ---------------------------------------------------------------------------
# Sizes
# ---------------------------------------------------------------------------
def sizes(M: int):
    nb = (M + 1) * (M + 2) // 2
    return dict(nb=nb, nst=nb * (M + 1), ne=2 * nb, nG=M + 1)


def recon_quad_n(M: int) -> int:
    """Duffy order for the reconstruction integrals: exact for degree M."""
    return (M + 3) // 2
