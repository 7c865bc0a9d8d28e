"""The ALE ADER-WENO finite volume scheme with local time stepping, written
plainly in FP64 NumPy (oracle, test infrastructure; never used by the product).

Paper: Boscheri, Dumbser, Zanotti, arXiv:1408.3719, Sec. 2.  Each function
names the passage it follows.  Batched functions work on arrays whose leading
axis runs over elements, edges or nodes; every batch member is independent.

Readings of points the paper leaves open (each one is also listed in the
design notes of the repository):
  R1  cycle semantics: the active set is taken from the cycle-start ticks; every
      node of an active element that lags behind its future time moves once;
      every edge with a moved node sweeps one bilinear space-time patch from
      its old to its new segment (edge fluxes and vertex fluxes of eq. eqn.STint
      in one form); the stages then run in the order of the algorithm
      description (motion, fluxes, update, projection, WENO, time step, predictor).
  R2  time steps are dyadic: a macro step spans 2^(L-1) nominal finest steps of
      theta (0.95) times the smallest CFL time step (eq. eqn.timestep) at its
      start and is cut into 2^30 integer ticks; an element steps the largest
      power of two of ticks within its CFL step, aligned to its current tick.
      Steps below the nominal finest one (2^(31-L) ticks) are taken when an
      element's CFL step falls below it during the macro step, so no step
      exceeds its element's CFL step.  L = 1 is global time stepping (theta 1).
  R3  the scheduling stencil is the symmetric closure of the WENO stencil and
      the vertex ring (so every predictor read lies inside its time slab).
  R4  predictor: only test functions with tau > 0 are kept in eq. CGfinal;
      M+1 Picard sweeps, per sweep V -> x -> metric -> P -> q; x_t from the
      isoparametric map; published velocity is v of the final iterate.
  R5  node velocity contributions of eq. NodesVel are time averages over
      [tau0, tau1]; masses use the element-stored area (eq. eqn.NScs.weights).
  R6  virtual geometry: element-stored vertices plus the exact time integral of
      the element's predicted vertex velocity; virtual average: reference mean
      of the predictor at tau; an element at the target time uses its real data.
  R7  constrained least squares: the element's own average is matched exactly,
      the others in the least-squares sense (unweighted).  The nonlinear weight
      omega_s of eq. weno is one scalar per stencil, shared by the four
      conserved variables, computed from the indicator summed over them.
  R10 boundaries: a transmissive edge takes as outer state the inner element's
      predicted cell mean at the flux point's time (a ghost copy of the
      element; the inner trace as outer state would leave the face without
      dissipation); slip walls mirror the normal momentum and their nodes slide
      along the (straight) wall.
  R8  lateral patch states: each element's predictor at the reference edge
      point chi and at the patch time rescaled to the element's time slab;
      Rusanov speed taken pointwise with the unnormalised normal.
  R9  memory variables are inflow-positive: Q^M_L -= G, Q^M_R += G, and
      |T'| Q' = |T| Q + Q^M; H^M tracks the space-time normal the same way.
  R11 Osher-type flux: 3 Gauss-Legendre points on the straight path; |A| by
      Sylvester's formula over the three distinct ALE wave speeds.
  R19 free local time steps (levels = 0, the paper's own LTS with each element
      at its CFL step, eq. eqn.timestep): the interval to the target time is one
      macro step of 2^30 ticks and an element steps floor(dt_CFL / delta) ticks
      (no power of two, no alignment), at most to the end of the interval; the
      update criterion eq. eqn.WENOupdate is then exact integer arithmetic.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import numpy as np

from . import euler
from . import tables as tb
from .topology import Topology, build_topology


@dataclasses.dataclass
class Config:
    M: int = 2
    gamma: float = 1.4
    cfl: float = 0.5
    levels: int = 1                   # L; 1 = global time stepping; 0 = free steps (FREE_TICKS)
    n_picard: int = 0                 # 0 -> M+1
    mesh_velocity: object = "lagrangian"   # "lagrangian" (V=v), "eulerian" (V=0) or callable V(x,y,t)
    weno_eps: float = 1e-14
    weno_r: float = 8.0
    weno_lambda: float = 1e5
    gcl_tol: float = 1e-12
    weno_shared: bool = True
    flux: str = "rusanov"             # "rusanov" (eq. eqn.rusanov), "osher" (eq. eqn.osher) or "hll"
    lts_fraction: float = 0.95        # nominal finest dyadic step / smallest CFL step (L >= 2)

    @property
    def npic(self):
        return self.n_picard if self.n_picard > 0 else self.M + 1


# ---------------------------------------------------------------------------
# Geometry helpers
# ---------------------------------------------------------------------------
def tri_area(X):
    """Signed area of triangles X (..., 3, 2)."""
    return 0.5 * ((X[..., 1, 0] - X[..., 0, 0]) * (X[..., 2, 1] - X[..., 0, 1])
                  - (X[..., 2, 0] - X[..., 0, 0]) * (X[..., 1, 1] - X[..., 0, 1]))


def tri_perimeter(X):
    acc = 0.0
    for k in range(3):
        d = X[..., (k + 1) % 3, :] - X[..., k, :]
        acc = acc + np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
    return acc


def affine_map(X, xi, eta):
    """x(xi, eta) of eq. xietaTransf for triangles X (..., 3, 2)."""
    xi = np.asarray(xi)
    eta = np.asarray(eta)
    return (X[..., 0, None, :] + (X[..., 1, None, :] - X[..., 0, None, :]) * xi[..., None]
            + (X[..., 2, None, :] - X[..., 0, None, :]) * eta[..., None])


def affine_inverse(X, x):
    """Reference coordinates of physical points x (..., P, 2) in triangles X (..., 3, 2)."""
    e1 = X[..., 1, :] - X[..., 0, :]
    e2 = X[..., 2, :] - X[..., 0, :]
    det = e1[..., 0] * e2[..., 1] - e2[..., 0] * e1[..., 1]
    d = x - X[..., 0, None, :]
    xi = (d[..., 0] * e2[..., 1, None] - d[..., 1] * e2[..., 0, None]) / det[..., None]
    eta = (e1[..., 0, None] * d[..., 1] - e1[..., 1, None] * d[..., 0]) / det[..., None]
    return xi, eta


# ---------------------------------------------------------------------------
# WENO reconstruction (eqs. intConsRec, weights, sigma, Sigma, eqn.weno)
# ---------------------------------------------------------------------------
def reconstruct_batch(M, cfg: Config, Xi, Qi, Xs, Qs, valid):
    """Polynomial WENO reconstruction on given (virtual) stencil data.

    Xi (Na,3,2), Qi (Na,4): element i at the reconstruction time (real data).
    Xs (Na,7,ne,3,2), Qs (Na,7,ne,4): stencil elements (virtual geometry and
    averages, eqs. eqn.virtGeom / eqn.virtCellaverage), entry 0 is i itself.
    valid (Na,7): stencil present.
    Returns (wnod (Na,nb,4) values at the nodal lattice, what (Na,nb,4) modal
    coefficients, wstencil (Na,7,nb,4), omega (Na,7,4)).
    """
    sz = tb.sizes(M)
    nb = sz["nb"]
    Na = Xi.shape[0]
    u, v, w = tb.duffy_rule(tb.recon_quad_n(M))
    wmean = w / w.sum()
    Sig = tb.sigma_matrix(M)
    what_s = np.zeros((Na, 7, nb, 4))
    sigma = np.zeros((Na, 7, 4))
    for s in range(7):
        ok = valid[:, s]
        if not ok.any():
            continue
        idx = np.nonzero(ok)[0]
        Xst = Xs[idx, s]                                  # (n, ne, 3, 2)
        xq = affine_map(Xst, u, v)                        # (n, ne, P, 2)
        Xii = Xi[idx][:, None]                            # (n, 1, 3, 2)
        xi, eta = affine_inverse(np.broadcast_to(Xii, Xst.shape), xq)
        A = np.einsum("njpl,p->njl", tb.eval_psi(M, xi, eta), wmean)   # means of psi_l over T~_j
        c = A[:, 0, :]                                    # constraint row (element i)
        b = Qs[idx, s]                                    # (n, ne, 4)
        # eliminate w_1 with the exact constraint c . w = Q_i
        Ar = A[:, 1:, 1:] - A[:, 1:, :1] * (c[:, None, 1:] / c[:, None, :1])
        br = b[:, 1:, :] - A[:, 1:, :1] * (Qi[idx][:, None, :] / c[:, None, :1])
        Qf, Rf = np.linalg.qr(Ar)                         # least squares by QR
        rest = np.linalg.solve(Rf, np.einsum("njk,njv->nkv", Qf, br))
        w0 = (Qi[idx] - np.einsum("nk,nkv->nv", c[:, 1:], rest)) / c[:, :1]
        ws = np.concatenate([w0[:, None, :], rest], axis=1)            # (n, nb, 4)
        what_s[idx, s] = ws
        sigma[idx, s] = np.einsum("nlv,lm,nmv->nv", ws, Sig, ws)
    lam = np.where(np.arange(7) == 0, cfg.weno_lambda, 1.0)
    if cfg.weno_shared:
        # one weight per stencil, shared by all variables (omega_s carries no variable index)
        sigma = np.repeat(sigma.sum(axis=2, keepdims=True), 4, axis=2)
    wt = lam[None, :, None] / (sigma + cfg.weno_eps) ** cfg.weno_r
    wt = np.where(valid[:, :, None], wt, 0.0)
    omega = wt / wt.sum(axis=1, keepdims=True)
    what = np.einsum("nsv,nslv->nlv", omega, what_s)
    psi_nodes = tb.eval_psi(M, tb.nodal_xy(M)[:, 0], tb.nodal_xy(M)[:, 1])   # (nb_nodes, nb)
    wnod = np.einsum("ml,nlv->nmv", psi_nodes, what)
    return wnod, what, what_s, omega


# ---------------------------------------------------------------------------
# Space-time Galerkin predictor (eqs. timeTransf .. newVertPos)
# ---------------------------------------------------------------------------
def predictor_batch(M, cfg: Config, wnod, Xe, dt, t0=None):
    """Element-local space-time predictor for the PDE and the mesh ODE.

    wnod (Na,nb,4): reconstruction at the nodal lattice at tau = 0.
    Xe (Na,3,2): element vertices at the current element time.
    dt (Na,): element time step.  t0 (Na,): physical start time (only used by
    a prescribed mesh velocity).
    Returns dict(avg (Na,M+1,4), trace (Na,3,nG,M+1,4), vvel (Na,3,M+1,2),
    q (Na,nb,M+1,4), x (Na,nb,M+1,2)).
    """
    nt = tb.nodal_tables(M)
    _, tm = tb.time_matrices(M)
    At, Bt, Dt = tm["At"], tm["Bt"], tm["Dt"]
    Dxi, Deta = nt["Dxi"], nt["Deta"]
    Na = wnod.shape[0]
    nodes = tb.nodal_xy(M)
    dt = np.asarray(dt, float)
    q = np.repeat(wnod[:, :, None, :], M + 1, axis=2).copy()            # (Na,nb,T,4)
    x0 = affine_map(Xe, nodes[:, 0], nodes[:, 1])                          # (Na,nb,2)
    x = np.repeat(x0[:, :, None, :], M + 1, axis=2).copy()               # (Na,nb,T,2)
    tnod = tb.time_nodes(M)

    def mesh_velocity(q, x):
        mv = cfg.mesh_velocity
        if isinstance(mv, str) and mv == "lagrangian":
            return q[..., 1:3] / q[..., 0:1]
        if isinstance(mv, str) and mv == "eulerian":
            return np.zeros(q.shape[:-1] + (2,))
        tt = t0[:, None, None] + dt[:, None, None] * tnod[None, None, :]
        return np.stack(mv(x[..., 0], x[..., 1], np.broadcast_to(tt, x.shape[:-1])), axis=-1)

    dtb = dt[:, None, None, None]
    for _ in range(cfg.npic):
        V = mesh_velocity(q, x)
        x[:, :, 1:, :] = (Bt[None, None, :, None] * x[:, :, 0:1, :]
                          + dtb * np.einsum("qr,nmrc->nmqc", At, V))
        x_xi = np.einsum("km,nmtc->nktc", Dxi, x)
        x_eta = np.einsum("km,nmtc->nktc", Deta, x)
        x_tau = np.einsum("pq,nmqc->nmpc", Dt, x)
        det = x_xi[..., 0] * x_eta[..., 1] - x_eta[..., 0] * x_xi[..., 1]
        xi_x = x_eta[..., 1] / det
        xi_y = -x_eta[..., 0] / det
        eta_x = -x_xi[..., 1] / det
        eta_y = x_xi[..., 0] / det
        xt = x_tau[..., 0] / dt[:, None, None]
        yt = x_tau[..., 1] / dt[:, None, None]
        xi_t = -(xi_x * xt + xi_y * yt)
        eta_t = -(eta_x * xt + eta_y * yt)
        f = euler.flux_f(q, cfg.gamma)
        g = euler.flux_g(q, cfg.gamma)
        dq_xi = np.einsum("km,nmtv->nktv", Dxi, q)
        dq_eta = np.einsum("km,nmtv->nktv", Deta, q)
        df_xi = np.einsum("km,nmtv->nktv", Dxi, f)
        df_eta = np.einsum("km,nmtv->nktv", Deta, f)
        dg_xi = np.einsum("km,nmtv->nktv", Dxi, g)
        dg_eta = np.einsum("km,nmtv->nktv", Deta, g)
        P = -(dq_xi * xi_t[..., None] + dq_eta * eta_t[..., None]
              + df_xi * xi_x[..., None] + df_eta * eta_x[..., None]
              + dg_xi * xi_y[..., None] + dg_eta * eta_y[..., None])          # eq. eqn.pdef, S = 0
        q[:, :, 1:, :] = (Bt[None, None, :, None] * q[:, :, 0:1, :]
                          + dtb * np.einsum("qr,nmrv->nmqv", At, P))
    V = mesh_velocity(q, x)
    vtx = tb.vertex_node_index(M)
    avg = np.einsum("m,nmtv->ntv", nt["amean"], q)
    trace = np.einsum("egm,nmtv->negtv", nt["edge"], q)
    vvel = V[:, vtx, :, :]
    return dict(avg=avg, trace=trace, vvel=vvel, q=q, x=x)


# ---------------------------------------------------------------------------
# Node solver NS_cs (eqs. eqnNScs, eqn.NScs.weights, eqn.dtau, NodesVel, eqn.newVertex)
# ---------------------------------------------------------------------------
def node_velocity(M, vvel_kj, tau0, tau1, mu):
    """Mass-weighted average of the element contributions to one node.
    vvel_kj (R, M+1, 2) vertex velocities of the ring elements at the node;
    tau0, tau1 (R,) rescaled node interval; mu (R,) masses.  Returns (2,)."""
    I = tb.lagrange_time_integral(M, tau0, tau1)                   # (R, M+1)
    vbar = np.einsum("rq,rqc->rc", I, vvel_kj) / (tau1 - tau0)[:, None]
    return (mu[:, None] * vbar).sum(axis=0) / mu.sum()


def wall_constraints(topo, X):
    """Unit outward normals of the slip walls at every node (zero off the
    walls) and a flag for nodes where two non-parallel walls meet (held fixed).
    Walls are straight, so the normals taken from the initial mesh stay valid."""
    nrm = np.zeros((topo.n_nodes, 2))
    pinned = np.zeros(topo.n_nodes, bool)
    for e in np.nonzero(topo.bc_tag == BC_SLIP)[0]:
        a, b = topo.edge_nodes[e]
        d = X[b] - X[a]
        n = np.array([d[1], -d[0]]) / np.hypot(d[0], d[1])
        for k in (a, b):
            if np.any(nrm[k] != 0) and abs(nrm[k, 0] * n[1] - nrm[k, 1] * n[0]) > 1e-9:
                pinned[k] = True
            nrm[k] = n
    return nrm, pinned


def wall_project(V, n, pinned):
    """Remove the wall-normal part of a node velocity (slip walls)."""
    if pinned:
        return np.zeros(2)
    return V - (V @ n) * n


# ---------------------------------------------------------------------------
# Space-time patch flux (eqs. eqn.spacetimenodes, G_ij, eqn.rusanov, A_n^V, eqn.STint)
# ---------------------------------------------------------------------------
def rusanov_flux(ql, qr, N, gamma):
    """Rusanov ALE flux through an unnormalised space-time normal N (..., 3)."""
    def ft(q):
        return (euler.flux_f(q, gamma) * N[..., 0:1] + euler.flux_g(q, gamma) * N[..., 1:2]
                + q * N[..., 2:3])

    nxy = np.sqrt(N[..., 0] ** 2 + N[..., 1] ** 2)

    def speed(q):
        rho, u, v, p = euler.primitives(q, gamma)
        return np.abs(u * N[..., 0] + v * N[..., 1] + N[..., 2]) + np.sqrt(gamma * p / rho) * nxy

    smax = np.maximum(speed(ql), speed(qr))
    return 0.5 * (ft(ql) + ft(qr)) - 0.5 * smax[..., None] * (qr - ql)


def _ale_flux_dot(q, N, gamma):
    """F~(q) . N = f N_x + g N_y + q N_t (eq. PDEdiv3D) for an unnormalised N."""
    return (euler.flux_f(q, gamma) * N[..., 0:1] + euler.flux_g(q, gamma) * N[..., 1:2]
            + q * N[..., 2:3])


def ale_jacobian(q, N, gamma):
    """d(F~(q) . N)/dq = A_x N_x + A_y N_y + N_t I, i.e. |N_xy| times the ALE
    Jacobian of eq. A_n^V along n = N_xy/|N_xy| with normal mesh speed
    -N_t/|N_xy|. A_x, A_y are the Jacobians of the Euler fluxes f and g written
    out from their definitions (eq. eulerTerms). Shape (..., 4, 4)."""
    rho, u, v, p = euler.primitives(q, gamma)
    gm = gamma - 1.0
    q2 = u * u + v * v
    H = (q[..., 3] + p) / rho
    z, o = np.zeros_like(u), np.ones_like(u)
    Ax = np.stack([
        np.stack([z, o, z, z], -1),
        np.stack([0.5 * gm * q2 - u * u, (3.0 - gamma) * u, -gm * v, gm * o], -1),
        np.stack([-u * v, v, u, z], -1),
        np.stack([u * (0.5 * gm * q2 - H), H - gm * u * u, -gm * u * v, gamma * u], -1)], -2)
    Ay = np.stack([
        np.stack([z, z, o, z], -1),
        np.stack([-u * v, v, u, z], -1),
        np.stack([0.5 * gm * q2 - v * v, -gm * u, (3.0 - gamma) * v, gm * o], -1),
        np.stack([v * (0.5 * gm * q2 - H), -gm * u * v, H - gm * v * v, gamma * v], -1)], -2)
    return (Ax * N[..., 0, None, None] + Ay * N[..., 1, None, None]
            + N[..., 2, None, None] * np.eye(4))


def ale_wave_speeds(q, N, gamma):
    """The three distinct eigenvalues of ale_jacobian: u.N_xy + N_t -/+ c |N_xy|
    and u.N_xy + N_t (a double one), shape (..., 3)."""
    rho, u, v, p = euler.primitives(q, gamma)
    un = u * N[..., 0] + v * N[..., 1] + N[..., 2]
    c = np.sqrt(gamma * p / rho) * np.sqrt(N[..., 0] ** 2 + N[..., 1] ** 2)
    return np.stack([un - c, un, un + c], -1)


def abs_matrix(A, lam):
    """|A| = R |Lambda| R^-1 (Sec. 2.4, after eq. eqn.path) for a diagonalizable A
    whose distinct eigenvalues are lam (..., 3), written without eigenvectors by
    Sylvester's formula: |A| = sum_k |lam_k| prod_{j != k} (A - lam_j I) / (lam_k - lam_j).
    Where the three coincide (N_xy = 0), A = lam I and |A| = |lam| I."""
    I = np.eye(4)
    out = np.zeros_like(A)
    spread = lam[..., 2] - lam[..., 0]
    ok = spread > 1e-300
    for k in range(3):
        term = np.broadcast_to(I, A.shape).copy()
        for j in range(3):
            if j != k:
                d = np.where(ok, lam[..., k] - lam[..., j], 1.0)
                term = term @ ((A - lam[..., j, None, None] * I) / d[..., None, None])
        out += np.abs(lam[..., k])[..., None, None] * term
    return np.where(ok[..., None, None], out, np.abs(lam[..., 1])[..., None, None] * I)


OSHER_POINTS = 3   # Gauss-Legendre points on the path (reading: the paper cites Gaussian quadrature)


def osher_flux(ql, qr, N, gamma, npts=OSHER_POINTS):
    """Osher-type ALE flux (eq. eqn.osher) with the straight-line path of eq.
    eqn.path, Psi(s) = ql + s (qr - ql), the path integral of |A| by Gauss-Legendre
    quadrature in s."""
    s, w = tb.gauss_legendre01(npts)
    dq = qr - ql
    D = np.zeros_like(dq)
    for k in range(npts):
        psi = ql + s[k] * dq
        A = ale_jacobian(psi, N, gamma)
        D += w[k] * np.einsum("...ij,...j->...i", abs_matrix(A, ale_wave_speeds(psi, N, gamma)), dq)
    return 0.5 * (_ale_flux_dot(ql, N, gamma) + _ale_flux_dot(qr, N, gamma)) - 0.5 * D


def hll_flux(ql, qr, N, gamma):
    """HLL ALE flux (not in the paper; an alternative dissipation): signal speeds
    of the ALE system along N, u.N_xy + N_t -/+ c |N_xy|, bounded over both
    states; upwind flux when both speeds have one sign."""
    nxy = np.sqrt(N[..., 0] ** 2 + N[..., 1] ** 2)

    def speeds(q):
        rho, u, v, p = euler.primitives(q, gamma)
        un = u * N[..., 0] + v * N[..., 1] + N[..., 2]
        c = np.sqrt(gamma * p / rho) * nxy
        return un - c, un + c

    l1, r1 = speeds(ql)
    l2, r2 = speeds(qr)
    sl, sr = np.minimum(l1, l2), np.maximum(r1, r2)
    fl, fr = _ale_flux_dot(ql, N, gamma), _ale_flux_dot(qr, N, gamma)
    den = np.where(sr > sl, sr - sl, 1.0)
    fh = (sr[..., None] * fl - sl[..., None] * fr + (sl * sr)[..., None] * (qr - ql)) / den[..., None]
    return np.where((sl >= 0)[..., None], fl, np.where((sr <= 0)[..., None], fr, fh))


FLUXES = {"rusanov": rusanov_flux, "osher": osher_flux, "hll": hll_flux}

BC_TRANSMISSIVE = 1
BC_SLIP = 2

# Ticks per macro step.  Free local time steps (paper-literal LTS, eq.
# eqn.timestep per element): one macro step covers the whole interval in 2^30
# ticks, and each element steps floor(dt_CFL / delta) ticks, so the update
# criterion stays integer arithmetic while every step is within 2^-30 of the
# interval below its CFL step.  Dyadic levels (R2): a macro step of L levels
# spans 2^(L-1) times the smallest CFL step at its start and is cut into the
# same 2^30 ticks, so the nominal finest step is 2^(31-L) ticks and the spare
# finer powers of two below it are there for elements whose CFL step falls
# below it during the macro step.
FREE_TICKS = 1 << 30
MACRO_TICKS = FREE_TICKS


def macro_tick(levels, dt_min, T, t_end, fraction=1.0):
    """Tick length of a macro step starting at time T: (t_end - T) / 2^30 for
    free steps; for L >= 1 levels, 2^(L-1) theta dt_min / 2^30 with the step
    fraction theta (1 for L = 1), clamped so that the macro step does not pass
    t_end (both divisions exact power-of-two scalings)."""
    rest = (t_end - T) / MACRO_TICKS
    if levels == 0:
        return rest
    theta = fraction if levels > 1 else 1.0
    return min((dt_min * theta) * ((1 << (levels - 1)) / MACRO_TICKS), rest)


def mirror_state(q, N):
    """Slip-wall ghost state: normal momentum reflected about the face normal."""
    nxy = np.sqrt(N[..., 0] ** 2 + N[..., 1] ** 2)
    nx, ny = N[..., 0] / nxy, N[..., 1] / nxy
    mn = q[..., 1] * nx + q[..., 2] * ny
    out = q.copy()
    out[..., 1] = q[..., 1] - 2.0 * mn * nx
    out[..., 2] = q[..., 2] - 2.0 * mn * ny
    return out


def patch_batch(M, cfg: Config, P, ticks, nL, sL, trL, nR, sR, trR, hasR, bc=None, avgL=None):
    """Flux and normal integral over bilinear space-time patches.

    P (E,4,3): corners (x, y, t) in the order old a, old b, new b, new a (eq.
    eqn.spacetimenodes); ticks (E,4) the same corners' tick times.
    nL, sL (E,): left element tick and step; trL (E,nG,M+1,4) its edge trace
    (chi running from a to b).  nR, sR, trR likewise for the right element,
    whose trace is read in reverse chi order; hasR (E,) False on boundary edges.
    bc (E,) boundary tag: a transmissive edge takes as outer state the inner
    element's predicted cell mean at the point's time (avgL (E,M+1,4), its
    means at the time nodes; R10), a slip wall the mirror image of the inner
    trace.
    Returns G (E,4) (outward from L) and Nint (E,3).
    """
    nG = M + 1
    chi, wc = tb.gauss_legendre01(nG)
    E = P.shape[0]
    G = np.zeros((E, 4))
    Nint = np.zeros((E, 3))
    P1, P2, P3, P4 = P[:, 0], P[:, 1], P[:, 2], P[:, 3]
    n1, n2, n3, n4 = ticks[:, 0], ticks[:, 1], ticks[:, 2], ticks[:, 3]
    for g in range(nG):
        for h in range(nG):
            c, t = chi[g], chi[h]
            dchi = (1 - t) * (P2 - P1) + t * (P3 - P4)
            dtau = (1 - c) * (P4 - P1) + c * (P3 - P2)
            N = np.cross(dchi, dtau)
            tk = (1 - c) * (1 - t) * n1 + c * (1 - t) * n2 + c * t * n3 + (1 - c) * t * n4
            lL = tb.lagrange_time(M, (tk - nL) / sL)
            ql = np.einsum("eq,eqv->ev", lL, trL[:, g])
            qr = ql.copy()
            slip = np.zeros(E, bool) if bc is None else (bc == BC_SLIP)
            if slip.any():
                qr = np.where(slip[:, None], mirror_state(ql, N), qr)
            open_ = ~hasR & ~slip
            if open_.any():
                if avgL is None:
                    raise ValueError("transmissive edges need the inner element's predicted means")
                qr = np.where(open_[:, None], np.einsum("eq,eqv->ev", lL, avgL), qr)
            if hasR.any():
                sRs = np.where(hasR, sR, 1)
                lR = tb.lagrange_time(M, (tk - nR) / sRs)
                qrr = np.einsum("eq,eqv->ev", lR, trR[:, nG - 1 - g])
                qr = np.where(hasR[:, None], qrr, qr)
            wgt = wc[g] * wc[h]
            G += wgt * FLUXES[cfg.flux](ql, qr, N, cfg.gamma)
            Nint += wgt * N
    return G, Nint


# ---------------------------------------------------------------------------
# Solver state
# ---------------------------------------------------------------------------
def level_step(dtcfl, delta, N, n, free):
    """Step in ticks of an element at tick n of a macro step of N ticks of
    length delta, and whether it overshoots its CFL step.
    Dyadic (R2): the largest power of two p <= N with p*delta <= dt_CFL,
    limited by the alignment of tick n; a tick is far below the nominal finest
    step, so p * delta > dt_CFL would need dt_CFL to fall below 2^-30 of the
    macro step.  Free (R19): floor(dt_CFL / delta), at most the ticks left.
    At least one tick."""
    if free:
        left = N - n
        q = dtcfl / delta
        p = left if q >= left else int(np.floor(q))
        return (1, True) if p < 1 else (p, False)
    p = N
    while p > 1 and p * delta > dtcfl:
        p //= 2
    over = p * delta > dtcfl
    if n > 0:
        p = min(p, n & (-n))
    return p, over


@dataclasses.dataclass
class State:
    Q: np.ndarray
    A: np.ndarray
    Xe: np.ndarray
    n: np.ndarray
    s: np.ndarray
    dtcfl: np.ndarray
    QM: np.ndarray
    HM: np.ndarray
    wnod: np.ndarray
    avg: np.ndarray
    trace: np.ndarray
    vvel: np.ndarray
    X: np.ndarray
    nk: np.ndarray
    T: float = 0.0
    delta: float = 0.0
    N: int = 1
    updates: int = 0
    node_moves: int = 0
    patches: int = 0
    cycles: int = 0
    macro_steps: int = 0
    cfl_overshoots: int = 0
    max_gcl: float = 0.0
    boundary_flux: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(4))
    active_sizes: list = dataclasses.field(default_factory=list)

    def copy(self):
        return dataclasses.replace(self, **{k: (v.copy() if isinstance(v, np.ndarray) else
                                                (list(v) if isinstance(v, list) else v))
                                            for k, v in dataclasses.asdict(self).items()})


class Solver:
    """Oracle solver: LTS cycles (R1, R2) on a moving triangular mesh."""

    def __init__(self, nodes, tris, Q0, cfg: Config, bedges=None, topo: Optional[Topology] = None):
        self.cfg = cfg
        M = cfg.M
        self.sz = tb.sizes(M)
        self.topo = topo if topo is not None else build_topology(nodes, tris, M, bedges)
        NE, NV = self.topo.n_elems, self.topo.n_nodes
        nb, nG = self.sz["nb"], self.sz["nG"]
        X = np.asarray(nodes, float).copy()
        Xe = X[self.topo.tris].copy()
        if (tri_area(Xe) <= 0).any():
            raise ValueError("mesh has non-positive (clockwise or degenerate) triangles")
        self.st = State(Q=np.asarray(Q0, float).copy(), A=tri_area(Xe), Xe=Xe,
                        n=np.zeros(NE, np.int64), s=np.zeros(NE, np.int64), dtcfl=np.zeros(NE),
                        QM=np.zeros((NE, 4)), HM=np.zeros((NE, 3)), wnod=np.zeros((NE, nb, 4)),
                        avg=np.zeros((NE, M + 1, 4)), trace=np.zeros((NE, 3, nG, M + 1, 4)),
                        vvel=np.zeros((NE, 3, M + 1, 2)), X=X, nk=np.zeros(NV, np.int64))
        self.st.N = MACRO_TICKS
        self.wall_n, self.wall_pin = wall_constraints(self.topo, X)
        # schedule record and override (parity tooling): step_log[i] lists the
        # steps element i took, in order; step_hook(i, k, p) may replace the
        # k-th step p that the level rule chose for element i
        self.step_log = [[] for _ in range(NE)]
        self.step_hook = None
        # delta_hook(m) may replace the tick length of macro step m (held fixed
        # when a schedule is replayed under perturbed data)
        self.delta_hook = None
        # pre-processing (Sec. 2.6): first reconstruction without projection and first CFL step
        allel = np.arange(NE)
        self._reconstruct(allel)
        self._local_dt(allel)
        self.fresh = True   # a macro boundary is pending (levels and predictors)

    # -- virtual projection (R6; eqs. eqn.virtGeom, eqn.virtCellaverage) ---------
    def _virtual(self, j, ntarget):
        """Geometry (...,3,2) and average (...,4) of elements j at tick ntarget."""
        st, M = self.st, self.cfg.M
        j = np.asarray(j)
        ntarget = np.broadcast_to(np.asarray(ntarget), j.shape)
        same = st.n[j] == ntarget
        if (~same & (st.s[j] <= 0)).any():
            raise AssertionError("projection of an element without a valid predictor")
        sj = np.where(same, 1, st.s[j])
        tau = np.where(same, 0.0, (ntarget - st.n[j]) / sj)
        dtj = sj * st.delta
        I = tb.lagrange_time_integral(M, np.zeros_like(tau), tau)              # (...,M+1)
        Xv = st.Xe[j] + dtj[..., None, None] * np.einsum("...q,...kqc->...kc", I, st.vvel[j])
        Qv = np.einsum("...q,...qv->...v", tb.lagrange_time(M, tau), st.avg[j])
        Xv = np.where(same[..., None, None], st.Xe[j], Xv)
        Qv = np.where(same[..., None], st.Q[j], Qv)
        return Xv, Qv

    def _reconstruct(self, elems):
        st, topo = self.st, self.topo
        if elems.size == 0:
            return
        sten = topo.stencils[elems]                              # (Na,7,ne)
        valid = sten[:, :, 0] >= 0
        sten_safe = np.where(sten >= 0, sten, elems[:, None, None])
        Xs, Qs = self._virtual(sten_safe, st.n[elems][:, None, None])
        wnod, _, _, _ = reconstruct_batch(self.cfg.M, self.cfg, st.Xe[elems], st.Q[elems], Xs, Qs, valid)
        st.wnod[elems] = wnod

    def _local_dt(self, elems):
        """eq. eqn.timestep over the element and its face neighbours (virtual data)."""
        st, topo = self.st, self.topo
        if elems.size == 0:
            return
        cand = np.concatenate([elems[:, None], topo.neigh[elems]], axis=1)    # (Na,4)
        ok = cand >= 0
        cs = np.where(ok, cand, elems[:, None])
        Xv, Qv = self._virtual(cs, st.n[elems][:, None])
        d = 4.0 * tri_area(Xv) / tri_perimeter(Xv)
        lam = euler.max_signal(Qv, self.cfg.gamma)
        ratio = np.where(ok, d / lam, np.inf)
        st.dtcfl[elems] = self.cfg.cfl * ratio.min(axis=1)

    def _level_step(self, elems):
        """Steps in ticks of the given elements (R2, R19), at least 1 (an
        overshoot of the CFL step is counted)."""
        st = self.st
        out = np.zeros(elems.size, np.int64)
        for t, i in enumerate(elems):
            p, over = level_step(st.dtcfl[i], st.delta, st.N, int(st.n[i]), self.cfg.levels == 0)
            if self.step_hook is not None:
                q = int(self.step_hook(int(i), len(self.step_log[i]), p))
                if q != p:
                    if not 1 <= q <= st.N - st.n[i]:
                        raise ValueError("a forced step must stay within the macro step")
                    p, over = q, q * st.delta > st.dtcfl[i]
            st.cfl_overshoots += over
            self.step_log[i].append(p)
            out[t] = p
        return out

    def _predict(self, elems):
        st = self.st
        if elems.size == 0:
            return
        dt = st.s[elems] * st.delta
        t0 = st.T + st.n[elems] * st.delta
        out = predictor_batch(self.cfg.M, self.cfg, st.wnod[elems], st.Xe[elems], dt, t0)
        st.avg[elems] = out["avg"]
        st.trace[elems] = out["trace"]
        st.vvel[elems] = out["vvel"]

    # -- macro-step boundary -----------------------------------------------------
    def macro_begin(self, t_end):
        st = self.st
        st.delta = macro_tick(self.cfg.levels, float(st.dtcfl.min()), st.T, t_end, self.cfg.lts_fraction)
        if self.delta_hook is not None:
            st.delta = float(self.delta_hook(st.macro_steps))
        allel = np.arange(self.topo.n_elems)
        st.n[:] = 0
        st.nk[:] = 0
        st.s[:] = self._level_step(allel)
        self._predict(allel)
        self.fresh = False

    # -- one cycle (R1) ----------------------------------------------------------
    def active_set(self):
        st, topo = self.st, self.topo
        fut = st.n + st.s
        act = []
        for i in range(topo.n_elems):
            if st.n[i] >= st.N:
                continue
            S = topo.sched[i]
            if st.n[S].max() <= fut[i] <= fut[S].min():
                act.append(i)
        return np.array(act, np.int64)

    def move_nodes(self, moved, newtick):
        """Node solver NS_cs (eqs. eqn.dtau, NodesVel, eqnNScs, eqn.NScs.weights,
        eqn.newVertex): each moved node k goes from its tick to newtick[k] with
        the mass-weighted time average of its ring elements' predicted vertex
        velocities; masses rho_j |T_j| from the element-stored state (R5).
        Returns the new node positions (the others unchanged)."""
        st, topo, M = self.st, self.topo, self.cfg.M
        Xnew = st.X.copy()
        for k in moved:
            ring = topo.ring[k]
            j = np.array([r[0] for r in ring])
            lv = np.array([r[1] for r in ring])
            if (st.s[j] <= 0).any():
                raise AssertionError("node ring element without a valid predictor")
            tau0 = (st.nk[k] - st.n[j]) / st.s[j]
            tau1 = (newtick[k] - st.n[j]) / st.s[j]
            mu = st.Q[j, 0] * st.A[j]
            V = node_velocity(M, st.vvel[j, lv], tau0, tau1, mu)
            V = wall_project(V, self.wall_n[k], self.wall_pin[k])
            Xnew[k] = st.X[k] + (newtick[k] - st.nk[k]) * st.delta * V
        return Xnew

    def cycle(self):
        st, topo, cfg, M = self.st, self.topo, self.cfg, self.cfg.M
        act = self.active_set()
        if act.size == 0:
            raise RuntimeError("deadlock: no element satisfies the update criterion")
        fut = st.n + st.s
        # nodes to move and their new ticks
        newtick = st.nk.copy()
        for i in act:
            for k in topo.tris[i]:
                if st.nk[k] < fut[i]:
                    if newtick[k] != st.nk[k] and newtick[k] != fut[i]:
                        raise AssertionError("co-active elements sharing a node disagree on its time")
                    newtick[k] = fut[i]
        moved = np.nonzero(newtick != st.nk)[0]
        Xnew = self.move_nodes(moved, newtick)
        # swept patches
        en = topo.edge_nodes
        is_moved = newtick != st.nk
        swept = np.nonzero(is_moved[en[:, 0]] | is_moved[en[:, 1]])[0]
        if swept.size:
            a, b = en[swept, 0], en[swept, 1]
            L, R = topo.edge_elems[swept, 0], topo.edge_elems[swept, 1]
            el, er = topo.edge_local[swept, 0], topo.edge_local[swept, 1]
            hasR = R >= 0
            Rs = np.where(hasR, R, L)
            ers = np.where(hasR, er, el)
            d = st.delta
            P = np.stack([
                np.concatenate([st.X[a], (st.nk[a] * d)[:, None]], 1),
                np.concatenate([st.X[b], (st.nk[b] * d)[:, None]], 1),
                np.concatenate([Xnew[b], (newtick[b] * d)[:, None]], 1),
                np.concatenate([Xnew[a], (newtick[a] * d)[:, None]], 1)], axis=1)
            ticks = np.stack([st.nk[a], st.nk[b], newtick[b], newtick[a]], 1).astype(float)
            if (st.s[L] <= 0).any() or (hasR & (st.s[Rs] <= 0)).any():
                raise AssertionError("patch neighbour without a valid predictor")
            G, Nint = patch_batch(M, cfg, P, ticks, st.n[L], st.s[L], st.trace[L, el],
                                  st.n[Rs], st.s[Rs], st.trace[Rs, ers], hasR,
                                  topo.bc_tag[swept], st.avg[L])
            # memory variables (eq. eqn.Qm2 and the geometric memory H^M), R9
            np.subtract.at(st.QM, L, G)
            np.subtract.at(st.HM, L, Nint)
            np.add.at(st.QM, R[hasR], G[hasR])
            np.add.at(st.HM, R[hasR], Nint[hasR])
            st.boundary_flux += G[~hasR].sum(axis=0)
        # conservative update of the active elements (eq. PDEfinal, S = 0)
        st.X = Xnew
        st.nk = newtick
        Xn = st.X[topo.tris[act]]
        An = tri_area(Xn)
        if not (An > 0).all():
            raise FloatingPointError("element inverted (or not finite) during the update")
        gcl = st.HM[act] - np.stack([np.zeros_like(An), np.zeros_like(An), An - st.A[act]], 1)
        rel = np.abs(gcl).max(axis=1) / (An + st.A[act])
        st.max_gcl = max(st.max_gcl, float(rel.max()))
        st.Q[act] = (st.A[act, None] * st.Q[act] + st.QM[act]) / An[:, None]
        _, _, _, pn = euler.primitives(st.Q[act], cfg.gamma)
        if not ((st.Q[act, 0] > 0).all() and (pn > 0).all()):
            raise FloatingPointError("non-physical state (rho <= 0, p <= 0 or not finite)")
        st.QM[act] = 0.0
        st.HM[act] = 0.0
        st.A[act] = An
        st.Xe[act] = Xn
        st.n[act] = fut[act]
        # projection + WENO, local time step, predictor for the next step
        self._reconstruct(act)
        self._local_dt(act)
        going = act[st.n[act] < st.N]
        done = act[st.n[act] >= st.N]
        st.s[done] = 0
        if going.size:
            st.s[going] = self._level_step(going)
            self._predict(going)
        st.updates += int(act.size)
        st.node_moves += int(moved.size)
        st.patches += int(swept.size)
        st.cycles += 1
        st.active_sizes.append(int(act.size))
        return act

    def macro_step(self, t_end):
        self.macro_begin(t_end)
        while (self.st.n < self.st.N).any():
            self.cycle()
        self.st.T = self.st.T + self.st.N * self.st.delta
        self.st.macro_steps += 1

    def run(self, t_end, max_macro_steps=None):
        k = 0
        while t_end - self.st.T > 1e-12 * max(1.0, abs(t_end)):
            if max_macro_steps is not None and k >= max_macro_steps:
                break
            self.macro_step(t_end)
            k += 1
        return self.st

    # -- diagnostics --------------------------------------------------------------
    def conserved_total(self):
        """sum_i (|T_i| Q_i + Q^M_i) + cumulative boundary outflow; constant in time."""
        st = self.st
        return (st.A[:, None] * st.Q + st.QM).sum(axis=0) + st.boundary_flux


# ---------------------------------------------------------------------------
# Global time stepping driver (separate code path, used to check LTS with L = 1)
# ---------------------------------------------------------------------------
def cfl_time_steps(Xe, Q, neigh, gamma, cfl):
    """Local CFL time step of eq. eqn.timestep with every element at one time:
    cfl * min over the element and its face neighbours of d / (|v| + c), with
    d the diameter of the inscribed circle, 4|T| / perimeter."""
    d = 4.0 * tri_area(Xe) / tri_perimeter(Xe)
    r = d / euler.max_signal(Q, gamma)
    rn = np.where(neigh >= 0, r[np.maximum(neigh, 0)], np.inf)
    return cfl * np.minimum(r, rn.min(axis=1))


class GTSSolver:
    """All elements advance together with dt = min CFL step: predictor on all,
    node motion on all nodes over [0,1], one patch per edge, direct update."""

    def __init__(self, nodes, tris, Q0, cfg: Config, bedges=None, topo=None):
        self.cfg = cfg
        self.topo = topo if topo is not None else build_topology(nodes, tris, cfg.M, bedges)
        self.X = np.asarray(nodes, float).copy()
        self.Q = np.asarray(Q0, float).copy()
        self.T = 0.0
        self.steps = 0
        self.wall_n, self.wall_pin = wall_constraints(self.topo, self.X)
        self._recon_dt()

    def _recon_dt(self):
        topo, cfg = self.topo, self.cfg
        Xe = self.X[topo.tris]
        sten = topo.stencils
        valid = sten[:, :, 0] >= 0
        ss = np.where(sten >= 0, sten, np.arange(topo.n_elems)[:, None, None])
        self.wnod, _, _, _ = reconstruct_batch(cfg.M, cfg, Xe, self.Q, Xe[ss], self.Q[ss], valid)
        self.dtcfl = cfl_time_steps(Xe, self.Q, topo.neigh, cfg.gamma, cfg.cfl)

    def step(self, t_end):
        topo, cfg, M = self.topo, self.cfg, self.cfg.M
        dt = min(float(self.dtcfl.min()), t_end - self.T)
        Xe = self.X[topo.tris]
        A = tri_area(Xe)
        pr = predictor_batch(M, cfg, self.wnod, Xe, np.full(topo.n_elems, dt),
                             np.full(topo.n_elems, self.T))
        Xn = self.X.copy()
        for k in range(topo.n_nodes):
            j = np.array([r[0] for r in topo.ring[k]])
            lv = np.array([r[1] for r in topo.ring[k]])
            V = node_velocity(M, pr["vvel"][j, lv], np.zeros(j.size), np.ones(j.size),
                              self.Q[j, 0] * A[j])
            Xn[k] = self.X[k] + dt * wall_project(V, self.wall_n[k], self.wall_pin[k])
        en = topo.edge_nodes
        a, b = en[:, 0], en[:, 1]
        L, R = topo.edge_elems[:, 0], topo.edge_elems[:, 1]
        el, er = topo.edge_local[:, 0], topo.edge_local[:, 1]
        hasR = R >= 0
        Rs = np.where(hasR, R, L)
        ers = np.where(hasR, er, el)
        z, o = np.zeros(a.size), np.full(a.size, dt)
        P = np.stack([np.column_stack([self.X[a], z]), np.column_stack([self.X[b], z]),
                      np.column_stack([Xn[b], o]), np.column_stack([Xn[a], o])], axis=1)
        ticks = np.tile(np.array([0.0, 0.0, 1.0, 1.0]), (a.size, 1))
        zero = np.zeros(a.size, np.int64)
        one = np.ones(a.size, np.int64)
        G, _ = patch_batch(M, cfg, P, ticks, zero, one, pr["trace"][L, el],
                           zero, one, pr["trace"][Rs, ers], hasR, topo.bc_tag, pr["avg"][L])
        flux = np.zeros((topo.n_elems, 4))
        np.add.at(flux, L, G)
        np.subtract.at(flux, R[hasR], G[hasR])
        An = tri_area(Xn[topo.tris])
        self.Q = (A[:, None] * self.Q - flux) / An[:, None]
        self.X = Xn
        self.T += dt
        self.steps += 1
        self._recon_dt()

    def run(self, t_end, max_steps=None):
        while t_end - self.T > 1e-12 * max(1.0, abs(t_end)):
            if max_steps is not None and self.steps >= max_steps:
                break
            self.step(t_end)
