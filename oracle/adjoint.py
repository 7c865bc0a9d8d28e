"""Reverse mode of one global time step (oracle, test infrastructure; never
used by the product): EulerianStep on a fixed mesh, LagrangianStep with the
mesh moving with the fluid (node positions differentiated as well).

The step is the scheme of Sec. 2 with one level (global time stepping) and the
mesh held fixed (Eulerian mode, V = 0 in eq. ODEmesh): WENO reconstruction
(eqs. intConsRec .. eqn.weno), space-time predictor (eq. CGfinal), Rusanov
(eq. eqn.rusanov) or HLL fluxes over the space-time faces (eq. eqn.STint) and
the one-step update (eq. PDEfinal), for a given time step dt that is held fixed
(the CFL step of eq. eqn.timestep is not differentiated).  It is written here
a second time with PyTorch CPU operations in FP64, following the NumPy oracle
step for step, so that torch.autograd yields the exact vector-Jacobian
product of the step map Q^n -> Q^{n+1}.

Everything that depends only on the fixed geometry (least-squares matrices of
the stencils, the metric of the reference maps, space-time normals, areas) is
computed once with the NumPy oracle's own tables and helpers; only the
dependence on the state runs through torch.

The forward map is pinned to the NumPy oracle's step and its derivative to
central differences of that step (tests/test_oracle_adjoint.py); the
Lagrangian step also to the translation invariance of the scheme.
"""
from __future__ import annotations

import numpy as np
import torch

from . import tables as tb
from .scheme import BC_SLIP, Config, affine_inverse, affine_map, tri_area
from .topology import build_topology

_F64 = torch.float64


def _t(a):
    return torch.as_tensor(np.asarray(a, np.float64), dtype=_F64)


def primitives(Q, gamma):
    """rho, u, v, p of eq. eqn.eos (same formula as the NumPy oracle)."""
    rho = Q[..., 0]
    u = Q[..., 1] / rho
    v = Q[..., 2] / rho
    p = (gamma - 1.0) * (Q[..., 3] - 0.5 * rho * (u * u + v * v))
    return rho, u, v, p


def flux_fg(Q, gamma):
    """Euler fluxes f and g of eq. eulerTerms."""
    rho, u, v, p = primitives(Q, gamma)
    E = Q[..., 3]
    f = torch.stack([rho * u, rho * u * u + p, rho * u * v, u * (E + p)], dim=-1)
    g = torch.stack([rho * v, rho * u * v, rho * v * v + p, v * (E + p)], dim=-1)
    return f, g


def rusanov(ql, qr, N, gamma):
    """Rusanov flux of eq. eqn.rusanov through an unnormalised space-time
    normal N; the larger signal speed is taken from the left state on ties and
    |x| has derivative sign(x) (0 at 0), fixing one subgradient."""
    nxy = torch.sqrt(N[..., 0] ** 2 + N[..., 1] ** 2)

    def ft(q):
        f, g = flux_fg(q, gamma)
        return f * N[..., 0:1] + g * N[..., 1:2] + q * N[..., 2:3]

    def speed(q):
        rho, u, v, p = primitives(q, gamma)
        return torch.abs(u * N[..., 0] + v * N[..., 1] + N[..., 2]) + torch.sqrt(gamma * p / rho) * nxy

    sl, sr = speed(ql), speed(qr)
    smax = torch.where(sl >= sr, sl, sr)
    return 0.5 * (ft(ql) + ft(qr)) - 0.5 * smax[..., None] * (qr - ql)


def hll(ql, qr, N, gamma):
    """HLL flux through an unnormalised space-time normal N (same formula as
    the NumPy oracle): signal speeds u.N_xy + N_t -/+ c|N_xy| bounded over both
    states, the left state's speed taken on ties; upwind when both speeds have
    one sign."""
    nxy = torch.sqrt(N[..., 0] ** 2 + N[..., 1] ** 2)

    def ft(q):
        f, g = flux_fg(q, gamma)
        return f * N[..., 0:1] + g * N[..., 1:2] + q * N[..., 2:3]

    def speeds(q):
        rho, u, v, p = primitives(q, gamma)
        un = u * N[..., 0] + v * N[..., 1] + N[..., 2]
        c = torch.sqrt(gamma * p / rho) * nxy
        return un - c, un + c

    l1, r1 = speeds(ql)
    l2, r2 = speeds(qr)
    sl = torch.where(l1 <= l2, l1, l2)
    sr = torch.where(r1 >= r2, r1, r2)
    fl, fr = ft(ql), ft(qr)
    den = torch.where(sr > sl, sr - sl, torch.ones_like(sr))
    fh = (sr[..., None] * fl - sl[..., None] * fr + (sl * sr)[..., None] * (qr - ql)) / den[..., None]
    return torch.where((sl >= 0)[..., None], fl, torch.where((sr <= 0)[..., None], fr, fh))


FLUX_FUNCTIONS = {"rusanov": rusanov, "hll": hll}


def mirror(q, N):
    """Slip-wall ghost state: normal momentum reflected (linear in q)."""
    nxy = torch.sqrt(N[..., 0] ** 2 + N[..., 1] ** 2)
    nx, ny = N[..., 0] / nxy, N[..., 1] / nxy
    mn = q[..., 1] * nx + q[..., 2] * ny
    return torch.stack([q[..., 0], q[..., 1] - 2.0 * mn * nx, q[..., 2] - 2.0 * mn * ny, q[..., 3]],
                       dim=-1)


class EulerianStep:
    """One global time step of length dt on a fixed mesh, as a torch function
    of the cell averages Q (NE, 4)."""

    def __init__(self, nodes, tris, cfg: Config, bedges=None, topo=None):
        if cfg.flux not in FLUX_FUNCTIONS:
            raise ValueError("the reverse-mode oracle covers the Rusanov and HLL fluxes")
        self.cfg = cfg
        M = cfg.M
        self.M = M
        self.topo = topo if topo is not None else build_topology(nodes, tris, M, bedges)
        topo = self.topo
        X = np.asarray(nodes, float)
        Xe = X[topo.tris]                                    # (NE,3,2)
        NE = topo.n_elems
        self.NE = NE
        self.area = tri_area(Xe)

        # -- reconstruction: constant least-squares maps per stencil (eq. intConsRec)
        sz = tb.sizes(M)
        nb = sz["nb"]
        u, v, w = tb.duffy_rule(tb.recon_quad_n(M))
        wmean = w / w.sum()
        sten = topo.stencils
        valid = sten[:, :, 0] >= 0
        ss = np.where(sten >= 0, sten, np.arange(NE)[:, None, None])
        self.sten_idx = torch.as_tensor(ss, dtype=torch.long)      # (NE,7,ne)
        self.valid = torch.as_tensor(valid)
        ne = ss.shape[2]
        Pm = np.zeros((NE, 7, nb - 1, ne - 1))   # rest = Pm @ br
        acol = np.zeros((NE, 7, ne - 1))         # A[1:, 0]
        cvec = np.ones((NE, 7, nb))              # constraint row c
        for s in range(7):
            idx = np.nonzero(valid[:, s])[0]
            if idx.size == 0:
                continue
            Xst = Xe[ss[idx, s]]
            xq = affine_map(Xst, u, v)
            Xii = Xe[idx][:, None]
            xi, eta = affine_inverse(np.broadcast_to(Xii, Xst.shape), xq)
            A = np.einsum("njpl,p->njl", tb.eval_psi(M, xi, eta), wmean)
            c = A[:, 0, :]
            Ar = A[:, 1:, 1:] - A[:, 1:, :1] * (c[:, None, 1:] / c[:, None, :1])
            Qf, Rf = np.linalg.qr(Ar)
            Pm[idx, s] = np.linalg.solve(Rf, np.transpose(Qf, (0, 2, 1)))
            acol[idx, s] = A[:, 1:, 0]
            cvec[idx, s] = c
        self.Pm, self.acol, self.cvec = _t(Pm), _t(acol), _t(cvec)
        self.Sig = _t(tb.sigma_matrix(M))
        self.lam = _t(np.where(np.arange(7) == 0, cfg.weno_lambda, 1.0))
        nxy = tb.nodal_xy(M)
        self.psi_nodes = _t(tb.eval_psi(M, nxy[:, 0], nxy[:, 1]))

        # -- predictor: constant metric of the fixed reference maps (eq. CGfinal, V = 0)
        nt = tb.nodal_tables(M)
        _, tm = tb.time_matrices(M)
        self.At, self.Bt, self.Dt = tm["At"], tm["Bt"], tm["Dt"]
        self.Dxi, self.Deta = _t(nt["Dxi"]), _t(nt["Deta"])
        self.edge_tab = _t(nt["edge"])
        self.amean = _t(nt["amean"])
        x0 = affine_map(Xe, nxy[:, 0], nxy[:, 1])                 # (NE,nb,2)
        x = np.repeat(x0[:, :, None, :], M + 1, axis=2).copy()
        x[:, :, 1:, :] = self.Bt[None, None, :, None] * x[:, :, 0:1, :]   # the motion ODE with V = 0
        self.x = x
        Dxi, Deta = nt["Dxi"], nt["Deta"]
        x_xi = np.einsum("km,nmtc->nktc", Dxi, x)
        x_eta = np.einsum("km,nmtc->nktc", Deta, x)
        det = x_xi[..., 0] * x_eta[..., 1] - x_eta[..., 0] * x_xi[..., 1]
        self.metric = dict(xi_x=x_eta[..., 1] / det, xi_y=-x_eta[..., 0] / det,
                           eta_x=-x_xi[..., 1] / det, eta_y=x_xi[..., 0] / det)
        self.x_tau = np.einsum("pq,nmqc->nmpc", self.Dt, x)

        # -- patches: fixed edges, corners (x, y, t) old a, old b, new b, new a
        en = topo.edge_nodes
        self.L = torch.as_tensor(topo.edge_elems[:, 0], dtype=torch.long)
        R = topo.edge_elems[:, 1]
        self.hasR = torch.as_tensor(R >= 0)
        self.Rs = torch.as_tensor(np.where(R >= 0, R, topo.edge_elems[:, 0]), dtype=torch.long)
        self.el = torch.as_tensor(topo.edge_local[:, 0], dtype=torch.long)
        self.ers = torch.as_tensor(np.where(R >= 0, topo.edge_local[:, 1], topo.edge_local[:, 0]),
                                   dtype=torch.long)
        self.slip = torch.as_tensor(topo.bc_tag == BC_SLIP)
        self.Xa, self.Xb = X[en[:, 0]], X[en[:, 1]]

    # ------------------------------------------------------------------
    def reconstruct(self, Q):
        """wnod (NE, nb, 4) of eq. eqn.weno from the averages Q (NE, 4)."""
        cfg = self.cfg
        Qs = Q[self.sten_idx]                                 # (NE,7,ne,4)
        Qi = Q[:, None, :]                                    # (NE,1,4)
        c0 = self.cvec[..., 0]                                # (NE,7)
        br = Qs[:, :, 1:, :] - self.acol[..., None] * (Qi[:, :, None, :] / c0[..., None, None])
        rest = torch.einsum("nskj,nsjv->nskv", self.Pm, br)   # (NE,7,nb-1,4)
        w0 = (Qi - torch.einsum("nsk,nskv->nsv", self.cvec[..., 1:], rest)) / c0[..., None]
        ws = torch.cat([w0[:, :, None, :], rest], dim=2)      # (NE,7,nb,4)
        sigma = torch.einsum("nslv,lm,nsmv->nsv", ws, self.Sig, ws)
        if cfg.weno_shared:
            sigma = sigma.sum(dim=2, keepdim=True).expand(-1, -1, 4)
        wt = self.lam[None, :, None] / (sigma + cfg.weno_eps) ** cfg.weno_r
        wt = torch.where(self.valid[:, :, None], wt, torch.zeros((), dtype=_F64))
        omega = wt / wt.sum(dim=1, keepdim=True)
        what = torch.einsum("nsv,nslv->nlv", omega, ws)
        return torch.einsum("ml,nlv->nmv", self.psi_nodes, what)

    def predict(self, wnod, dt):
        """Edge traces (NE, 3, nG, M+1, 4) and cell means at the time nodes
        (NE, M+1, 4) of the space-time predictor with the tau = 0 data fixed
        (eq. CGfinal), M+1 (or n_picard) Picard sweeps."""
        M, cfg = self.M, self.cfg
        T = M + 1
        met = {k: _t(v)[..., None] for k, v in self.metric.items()}
        xt = _t(self.x_tau[..., 0] / dt)
        yt = _t(self.x_tau[..., 1] / dt)
        xi_t = -(met["xi_x"][..., 0] * xt + met["xi_y"][..., 0] * yt)[..., None]
        eta_t = -(met["eta_x"][..., 0] * xt + met["eta_y"][..., 0] * yt)[..., None]
        At, Bt = _t(self.At), _t(self.Bt)
        q = wnod[:, :, None, :].expand(-1, -1, T, -1)
        for _ in range(cfg.npic):
            f, g = flux_fg(q, cfg.gamma)
            d = lambda D, a: torch.einsum("km,nmtv->nktv", D, a)   # noqa: E731
            P = -(d(self.Dxi, q) * xi_t + d(self.Deta, q) * eta_t
                  + d(self.Dxi, f) * met["xi_x"] + d(self.Deta, f) * met["eta_x"]
                  + d(self.Dxi, g) * met["xi_y"] + d(self.Deta, g) * met["eta_y"])
            upper = (Bt[None, None, :, None] * q[:, :, 0:1, :]
                     + dt * torch.einsum("qr,nmrv->nmqv", At, P))
            q = torch.cat([q[:, :, 0:1, :], upper], dim=2)
        return (torch.einsum("egm,nmtv->negtv", self.edge_tab, q),
                torch.einsum("m,nmtv->ntv", self.amean, q))

    def fluxes(self, trace, avg, dt):
        """Edge fluxes G (NF, 4), outward from L, over the space-time faces of
        the fixed edges (eq. eqn.STint with (M+1)^2 Gauss points); transmissive
        edges take the inner element's predicted mean as outer state (R10)."""
        M, cfg = self.M, self.cfg
        nG = M + 1
        chi, wc = tb.gauss_legendre01(nG)
        z = np.zeros(self.Xa.shape[0])
        P1 = np.column_stack([self.Xa, z])
        P2 = np.column_stack([self.Xb, z])
        P3 = np.column_stack([self.Xb, z + dt])
        P4 = np.column_stack([self.Xa, z + dt])
        trL = trace[self.L, self.el]                          # (NF,nG,T,4)
        trR = trace[self.Rs, self.ers]
        avL = avg[self.L]                                     # (NF,T,4)
        G = torch.zeros((self.Xa.shape[0], 4), dtype=_F64)
        for g in range(nG):
            for h in range(nG):
                c, t = chi[g], chi[h]
                dchi = (1 - t) * (P2 - P1) + t * (P3 - P4)
                dtau = (1 - c) * (P4 - P1) + c * (P3 - P2)
                N = _t(np.cross(dchi, dtau))
                tk = (1 - c) * (1 - t) * 0.0 + c * (1 - t) * 0.0 + c * t * 1.0 + (1 - c) * t * 1.0
                lt = _t(tb.lagrange_time(M, np.array([tk]))[0])
                ql = torch.einsum("q,eqv->ev", lt, trL[:, g])
                qrr = torch.einsum("q,eqv->ev", lt, trR[:, nG - 1 - g])
                qr = torch.where(self.slip[:, None], mirror(ql, N),
                                 torch.einsum("q,eqv->ev", lt, avL))
                qr = torch.where(self.hasR[:, None], qrr, qr)
                G = G + (wc[g] * wc[h]) * FLUX_FUNCTIONS[cfg.flux](ql, qr, N, cfg.gamma)
        return G

    def __call__(self, Q, dt):
        """Q^{n+1} from Q^n (torch (NE, 4)) for the fixed step dt."""
        trace, avg = self.predict(self.reconstruct(Q), dt)
        G = self.fluxes(trace, avg, dt)
        flux = torch.zeros_like(Q).index_add(0, self.L, G)
        flux = flux.index_add(0, self.Rs[self.hasR], -G[self.hasR])
        A = _t(self.area)[:, None]
        return (A * Q - flux) / A

    def vjp(self, Q, dt, Qbar_next):
        """(dQ^{n+1}/dQ^n)^T Qbar_next, NumPy in and out."""
        q = _t(Q).requires_grad_(True)
        out = self(q, dt)
        (g,) = torch.autograd.grad(out, q, _t(Qbar_next))
        return g.detach().numpy()

    def step(self, Q, dt):
        with torch.no_grad():
            return self(_t(Q), dt).numpy()


# ---------------------------------------------------------------------------
# Lagrangian global step: state and node positions both differentiated
# ---------------------------------------------------------------------------
def _tri_area_t(X):
    return 0.5 * ((X[..., 1, 0] - X[..., 0, 0]) * (X[..., 2, 1] - X[..., 0, 1])
                  - (X[..., 2, 0] - X[..., 0, 0]) * (X[..., 1, 1] - X[..., 0, 1]))


def _affine_map_t(X, xi, eta):
    """x(xi, eta) of eq. xietaTransf for triangles X (..., 3, 2) at constant
    reference points (P,) -> (..., P, 2)."""
    return (X[..., 0, None, :] + (X[..., 1, None, :] - X[..., 0, None, :]) * xi[:, None]
            + (X[..., 2, None, :] - X[..., 0, None, :]) * eta[:, None])


def _affine_inverse_t(X, x):
    """Reference coordinates of points x (..., P, 2) in triangles X (..., 3, 2)."""
    e1 = X[..., 1, :] - X[..., 0, :]
    e2 = X[..., 2, :] - X[..., 0, :]
    det = e1[..., 0] * e2[..., 1] - e2[..., 0] * e1[..., 1]
    d = x - X[..., 0, None, :]
    xi = (d[..., 0] * e2[..., 1, None] - d[..., 1] * e2[..., 0, None]) / det[..., None]
    eta = (e1[..., 0, None] * d[..., 1] - e1[..., 1, None] * d[..., 0]) / det[..., None]
    return xi, eta


class LagrangianStep:
    """One global time step of length dt with the mesh moving with the fluid
    (Lagrangian mode, V = v in eq. ODEmesh), as a torch function of the cell
    averages Q (NE, 4) and the node positions X (NV, 2): the reconstruction on
    the current geometry (eqs. intConsRec .. eqn.weno), the predictor of the
    PDE and the mesh ODE (eqs. CGfinal, VCG, newVertPos), the node solver
    (eqs. eqnNScs, eqn.NScs.weights, NodesVel, eqn.newVertex over [0, 1]), the
    fluxes over the bilinear space-time patches of the moving edges (eqs.
    eqn.spacetimenodes, G_ij, eqn.STint) and the update with the new areas
    (eq. PDEfinal). Every geometric quantity is computed from X inside the
    graph, so torch.autograd gives the vector-Jacobian product with respect to
    both Q and X (dt held fixed)."""

    def __init__(self, nodes, tris, cfg: Config, bedges=None, topo=None):
        if cfg.flux not in FLUX_FUNCTIONS:
            raise ValueError("the reverse-mode oracle covers the Rusanov and HLL fluxes")
        if cfg.mesh_velocity not in ("lagrangian", "eulerian"):
            raise ValueError("a prescribed mesh velocity is not covered")
        from .scheme import wall_constraints
        self.cfg = cfg
        # V = v (the mesh moves with the fluid) or V = 0 (a fixed mesh, eq. ODEmesh)
        self.vscale = 1.0 if cfg.mesh_velocity == "lagrangian" else 0.0
        M = cfg.M
        self.M = M
        self.topo = topo if topo is not None else build_topology(nodes, tris, M, bedges)
        topo = self.topo
        self.NE, self.NV = topo.n_elems, topo.n_nodes
        self.tris = torch.as_tensor(topo.tris, dtype=torch.long)
        sten = topo.stencils
        self.valid = sten[:, :, 0] >= 0
        self.sten = sten
        # reference-element tables (constants)
        u, v, w = tb.duffy_rule(tb.recon_quad_n(M))
        self.qu, self.qv, self.qw = _t(u), _t(v), _t(w / w.sum())
        self.mons = tb.monomials(M)
        self.psiC = _t(tb.psi_coeffs(M))                      # (nb, n_mono)
        self.Sig = _t(tb.sigma_matrix(M))
        self.lam = _t(np.where(np.arange(7) == 0, cfg.weno_lambda, 1.0))
        nxy = tb.nodal_xy(M)
        self.nod_xi, self.nod_eta = _t(nxy[:, 0]), _t(nxy[:, 1])
        self.psi_nodes = _t(tb.eval_psi(M, nxy[:, 0], nxy[:, 1]))
        nt = tb.nodal_tables(M)
        _, tm = tb.time_matrices(M)
        self.At, self.Bt, self.Dt = _t(tm["At"]), _t(tm["Bt"]), _t(tm["Dt"])
        self.Dxi, self.Deta = _t(nt["Dxi"]), _t(nt["Deta"])
        self.edge_tab = _t(nt["edge"])
        self.amean = _t(nt["amean"])
        self.vtx = torch.as_tensor(tb.vertex_node_index(M), dtype=torch.long)
        self.Iq = _t(tb.lagrange_time_integral(M, 0.0, 1.0))  # time averages over [0, 1]
        # node rings and slip walls
        ring = [(k, j, lv) for k in range(self.NV) for (j, lv) in topo.ring[k]]
        self.r_node = torch.as_tensor([r[0] for r in ring], dtype=torch.long)
        self.r_elem = torch.as_tensor([r[1] for r in ring], dtype=torch.long)
        self.r_lv = torch.as_tensor([r[2] for r in ring], dtype=torch.long)
        wn, pin = wall_constraints(topo, np.asarray(nodes, float))
        self.wall_n = _t(wn)
        self.wall_free = _t((~pin).astype(float))
        # edges
        en = topo.edge_nodes
        self.ea = torch.as_tensor(en[:, 0], dtype=torch.long)
        self.eb = torch.as_tensor(en[:, 1], dtype=torch.long)
        self.L = torch.as_tensor(topo.edge_elems[:, 0], dtype=torch.long)
        R = topo.edge_elems[:, 1]
        self.hasR = torch.as_tensor(R >= 0)
        self.Rs = torch.as_tensor(np.where(R >= 0, R, topo.edge_elems[:, 0]), dtype=torch.long)
        self.el = torch.as_tensor(topo.edge_local[:, 0], dtype=torch.long)
        self.ers = torch.as_tensor(np.where(R >= 0, topo.edge_local[:, 1], topo.edge_local[:, 0]),
                                   dtype=torch.long)
        self.slip = torch.as_tensor(topo.bc_tag == BC_SLIP)

    def _psi(self, xi, eta):
        mono = torch.stack([xi ** a * eta ** b for (a, b) in self.mons], dim=-1)
        return mono @ self.psiC.T

    def reconstruct(self, Q, Xe):
        """wnod (NE, nb, 4) on the current geometry Xe (NE, 3, 2)."""
        ss = torch.as_tensor(np.where(self.sten >= 0, self.sten, np.arange(self.NE)[:, None, None]),
                             dtype=torch.long)
        return self.recon_core(Xe, Q, Xe[ss], Q[ss], self.valid)

    def recon_core(self, Xi, Qi_all, Xs, Qs, valid_np):
        """wnod (n, nb, 4) of elements with vertices Xi (n, 3, 2) and averages
        Qi_all (n, 4), their stencils' elements given as Xs (n, 7, ne, 3, 2)
        and Qs (n, 7, ne, 4) (row 0 the element itself; real or projected
        data), valid_np (n, 7) the stencils that exist."""
        cfg, n_el = self.cfg, Xi.shape[0]
        nb = self.psiC.shape[0]
        ws_all = torch.zeros((n_el, 7, nb, 4), dtype=_F64)
        sig_all = torch.zeros((n_el, 7, 4), dtype=_F64)
        for s in range(7):
            idx_np = np.nonzero(valid_np[:, s])[0]
            if idx_np.size == 0:
                continue
            idx = torch.as_tensor(idx_np, dtype=torch.long)
            Xst = Xs[idx, s]                                                      # (n, ne, 3, 2)
            xq = _affine_map_t(Xst, self.qu, self.qv)                             # (n, ne, P, 2)
            Xii = Xi[idx][:, None].expand_as(Xst)
            xi, eta = _affine_inverse_t(Xii, xq)
            A = torch.einsum("njpl,p->njl", self._psi(xi, eta), self.qw)         # (n, ne, nb)
            c = A[:, 0, :]
            Qi = Qi_all[idx]
            b = Qs[idx, s]                                                        # (n, ne, 4)
            Ar = A[:, 1:, 1:] - A[:, 1:, :1] * (c[:, None, 1:] / c[:, None, :1])
            br = b[:, 1:, :] - A[:, 1:, :1] * (Qi[:, None, :] / c[:, None, :1])
            Qf, Rf = torch.linalg.qr(Ar)
            rest = torch.linalg.solve_triangular(Rf, Qf.transpose(1, 2) @ br, upper=True)
            w0 = (Qi - torch.einsum("nk,nkv->nv", c[:, 1:], rest)) / c[:, :1]
            ws = torch.cat([w0[:, None, :], rest], dim=1)                         # (n, nb, 4)
            sig = torch.einsum("nlv,lm,nmv->nv", ws, self.Sig, ws)
            ws_all = ws_all.index_put((idx, torch.full_like(idx, s)), ws)
            sig_all = sig_all.index_put((idx, torch.full_like(idx, s)), sig)
        valid = torch.as_tensor(valid_np)
        if cfg.weno_shared:
            sig_all = sig_all.sum(dim=2, keepdim=True).expand(-1, -1, 4)
        wt = self.lam[None, :, None] / (sig_all + cfg.weno_eps) ** cfg.weno_r
        wt = torch.where(valid[:, :, None], wt, torch.zeros((), dtype=_F64))
        omega = wt / wt.sum(dim=1, keepdim=True)
        what = torch.einsum("nsv,nslv->nlv", omega, ws_all)
        return torch.einsum("ml,nlv->nmv", self.psi_nodes, what)

    def predict(self, wnod, Xe, dt):
        """Space-time predictor with the mesh moving at the fluid velocity:
        traces (NE, 3, nG, T, 4), means (NE, T, 4), vertex velocities (NE, 3, T, 2).
        dt: one step for all elements, or one per element."""
        M, cfg = self.M, self.cfg
        T = M + 1
        if np.ndim(dt):
            dt = _t(dt)[:, None, None]
            dt4 = dt[..., None]
        else:
            dt4 = dt
        q = wnod[:, :, None, :].expand(-1, -1, T, -1)
        x0 = _affine_map_t(Xe, self.nod_xi, self.nod_eta)                        # (NE, nb, 2)
        x = x0[:, :, None, :].expand(-1, -1, T, -1)
        d = lambda D, a: torch.einsum("km,nmtv->nktv", D, a)   # noqa: E731
        for _ in range(cfg.npic):
            V = self.vscale * (q[..., 1:3] / q[..., 0:1])
            xu = self.Bt[None, None, :, None] * x[:, :, 0:1, :] + dt4 * torch.einsum("qr,nmrc->nmqc", self.At, V)
            x = torch.cat([x[:, :, 0:1, :], xu], dim=2)
            x_xi, x_eta = d(self.Dxi, x), d(self.Deta, x)
            x_tau = torch.einsum("pq,nmqc->nmpc", self.Dt, x)
            det = x_xi[..., 0] * x_eta[..., 1] - x_eta[..., 0] * x_xi[..., 1]
            xi_x, xi_y = x_eta[..., 1] / det, -x_eta[..., 0] / det
            eta_x, eta_y = -x_xi[..., 1] / det, x_xi[..., 0] / det
            xt, yt = x_tau[..., 0] / dt, x_tau[..., 1] / dt
            xi_t = -(xi_x * xt + xi_y * yt)
            eta_t = -(eta_x * xt + eta_y * yt)
            f, g = flux_fg(q, cfg.gamma)
            P = -(d(self.Dxi, q) * xi_t[..., None] + d(self.Deta, q) * eta_t[..., None]
                  + d(self.Dxi, f) * xi_x[..., None] + d(self.Deta, f) * eta_x[..., None]
                  + d(self.Dxi, g) * xi_y[..., None] + d(self.Deta, g) * eta_y[..., None])
            qu = self.Bt[None, None, :, None] * q[:, :, 0:1, :] + dt4 * torch.einsum("qr,nmrv->nmqv", self.At, P)
            q = torch.cat([q[:, :, 0:1, :], qu], dim=2)
        V = self.vscale * (q[..., 1:3] / q[..., 0:1])
        return (torch.einsum("egm,nmtv->negtv", self.edge_tab, q),
                torch.einsum("m,nmtv->ntv", self.amean, q), V[:, self.vtx])

    def move_nodes(self, X, Q, A, vvel, dt):
        """New node positions: mass-weighted (rho |T|) mean over each node's ring
        of the vertex velocities averaged over [0, 1]; slip-wall nodes slide."""
        vbar = torch.einsum("q,rqc->rc", self.Iq, vvel[self.r_elem, self.r_lv])
        mu = (Q[:, 0] * A)[self.r_elem]
        num = torch.zeros((self.NV, 2), dtype=_F64).index_add(0, self.r_node, mu[:, None] * vbar)
        den = torch.zeros(self.NV, dtype=_F64).index_add(0, self.r_node, mu)
        V = num / den[:, None]
        V = (V - (V * self.wall_n).sum(dim=1, keepdim=True) * self.wall_n) * self.wall_free[:, None]
        return X + dt * V

    def fluxes(self, X, Xn, trace, avg, dt):
        M, cfg = self.M, self.cfg
        nG = M + 1
        chi, wc = tb.gauss_legendre01(nG)
        NF = self.ea.shape[0]
        z = torch.zeros((NF, 1), dtype=_F64)
        P1 = torch.cat([X[self.ea], z], 1)
        P2 = torch.cat([X[self.eb], z], 1)
        P3 = torch.cat([Xn[self.eb], z + dt], 1)
        P4 = torch.cat([Xn[self.ea], z + dt], 1)
        trL = trace[self.L, self.el]
        trR = trace[self.Rs, self.ers]
        avL = avg[self.L]
        G = torch.zeros((NF, 4), dtype=_F64)
        for g in range(nG):
            for h in range(nG):
                c, t = float(chi[g]), float(chi[h])
                dchi = (1 - t) * (P2 - P1) + t * (P3 - P4)
                dtau = (1 - c) * (P4 - P1) + c * (P3 - P2)
                N = torch.linalg.cross(dchi, dtau, dim=-1)
                lt = _t(tb.lagrange_time(M, np.array([t]))[0])
                ql = torch.einsum("q,eqv->ev", lt, trL[:, g])
                qrr = torch.einsum("q,eqv->ev", lt, trR[:, nG - 1 - g])
                qr = torch.where(self.slip[:, None], mirror(ql, N), torch.einsum("q,eqv->ev", lt, avL))
                qr = torch.where(self.hasR[:, None], qrr, qr)
                G = G + (wc[g] * wc[h]) * FLUX_FUNCTIONS[cfg.flux](ql, qr, N, cfg.gamma)
        return G

    def __call__(self, Q, X, dt):
        """(Q^{n+1}, X^{n+1}) from (Q^n, X^n) for the fixed step dt."""
        Xe = X[self.tris]
        A = _tri_area_t(Xe)
        trace, avg, vvel = self.predict(self.reconstruct(Q, Xe), Xe, dt)
        Xn = self.move_nodes(X, Q, A, vvel, dt)
        G = self.fluxes(X, Xn, trace, avg, dt)
        flux = torch.zeros_like(Q).index_add(0, self.L, G)
        flux = flux.index_add(0, self.Rs[self.hasR], -G[self.hasR])
        An = _tri_area_t(Xn[self.tris])
        return (A[:, None] * Q - flux) / An[:, None], Xn

    def vjp(self, Q, X, dt, Qbar_next, Xbar_next):
        """Adjoints (Qbar, Xbar) of (Q^n, X^n) for (Qbar_next, Xbar_next) of
        (Q^{n+1}, X^{n+1}); NumPy in and out."""
        q = _t(Q).requires_grad_(True)
        x = _t(X).requires_grad_(True)
        qn, xn = self(q, x, dt)
        gq, gx = torch.autograd.grad((qn, xn), (q, x), (_t(Qbar_next), _t(Xbar_next)))
        return gq.detach().numpy(), gx.detach().numpy()

    def step(self, Q, X, dt):
        with torch.no_grad():
            qn, xn = self(_t(Q), _t(X), dt)
        return qn.numpy(), xn.numpy()


# ---------------------------------------------------------------------------
# Dyadic LTS macro step with its schedule frozen (mesh moving with the fluid)
# ---------------------------------------------------------------------------
def lts_schedule(solver, t_end, n_macro):
    """Advance the NumPy LTS oracle `solver` by n_macro macro steps and return
    what it decided: per macro step the tick length delta and, per element,
    the steps (in ticks) it took, in order."""
    out = []
    for _ in range(n_macro):
        before = [len(x) for x in solver.step_log]
        solver.macro_step(t_end)
        out.append((solver.st.delta, [solver.step_log[i][before[i]:] for i in range(len(before))]))
    return out


class LagrangianLTS:
    """Macro steps of the local time stepping scheme (Sec. 2.6: dyadic levels or
    free steps (levels = 0: one macro step of 2^30 ticks to the target time),
    the update criterion over the scheduling stencil, virtual projection of
    the stencil in space and time, eqs. eqn.virtGeom and eqn.virtCellaverage;
    the node solver over each node's own interval, eqs. eqn.dtau .. eqn.newVertex;
    swept space-time patches with corners at different times, eqs.
    eqn.spacetimenodes and eqn.STint; memory variables, eq. eqn.Qm2) with the
    mesh moving with the fluid (or held fixed: V = 0), written with PyTorch CPU operations in FP64
    after the NumPy oracle's Solver, cycle by cycle, with the schedule held
    fixed: the tick length of every macro step and every element's sequence of
    steps are inputs (taken from a run of the NumPy oracle), so the update
    sets, node and patch sets follow from integer ticks alone and the map
    (Q, X, wnod) -> (Q', X', wnod') over a macro step is smooth where its
    fluxes and WENO weights are. The state between macro steps is the
    averages, the node positions and each element's last reconstruction
    (nodal values wnod): element vertices and areas then follow from X."""

    def __init__(self, nodes, tris, cfg: Config, bedges=None, topo=None):
        self.g = LagrangianStep(nodes, tris, cfg, bedges=bedges, topo=topo)
        g = self.g
        self.cfg, self.M, self.topo = cfg, cfg.M, g.topo
        self.NE, self.NV = g.NE, g.NV
        self.sten = g.sten
        self.r_node = g.r_node.numpy()
        self.r_elem = g.r_elem.numpy()
        self.r_lv = g.r_lv.numpy()

    # -- pieces of a cycle ------------------------------------------------------
    def _virtual(self, j, ntarget, Q, Xe, avg, vvel, n, s, delta):
        """Vertices (..., 3, 2) and average (..., 4) of elements j projected to
        tick ntarget with their predictors; real data where the ticks agree."""
        M = self.M
        same = n[j] == ntarget
        sj = np.where(same, 1, s[j])
        tau = np.where(same, 0.0, (ntarget - n[j]) / sj)
        dtj = sj * delta
        I = _t(tb.lagrange_time_integral(M, np.zeros_like(tau), tau))
        lt = _t(tb.lagrange_time(M, tau))
        jt = torch.as_tensor(j, dtype=torch.long)
        Xv = Xe[jt] + _t(dtj)[..., None, None] * torch.einsum("...q,...kqc->...kc", I, vvel[jt])
        Qv = torch.einsum("...q,...qv->...v", lt, avg[jt])
        sm = torch.as_tensor(same)
        return (torch.where(sm[..., None, None], Xe[jt], Xv), torch.where(sm[..., None], Q[jt], Qv))

    def _reconstruct(self, act, Q, Xe, avg, vvel, n, s, delta):
        sten = self.sten[act]
        valid = sten[:, :, 0] >= 0
        ss = np.where(sten >= 0, sten, act[:, None, None])
        nt = np.broadcast_to(n[act][:, None, None], ss.shape)
        Xs, Qs = self._virtual(ss, nt, Q, Xe, avg, vvel, n, s, delta)
        ta = torch.as_tensor(act, dtype=torch.long)
        return self.g.recon_core(Xe[ta], Q[ta], Xs, Qs, valid)

    def _move(self, X, Q, A, vvel, n, s, nk, newtick, moved, delta):
        """New node positions: each moved node over its own interval [nk, newtick]
        with the mass-weighted mean of its ring's vertex velocities averaged over
        that interval of each ring element's predictor."""
        if moved.size == 0:
            return X
        g, M = self.g, self.M
        sel = np.isin(self.r_node, moved)
        rk, rj, rl = self.r_node[sel], self.r_elem[sel], self.r_lv[sel]
        if (s[rj] <= 0).any():
            raise AssertionError("node ring element without a valid predictor")
        tau0 = (nk[rk] - n[rj]) / s[rj]
        tau1 = (newtick[rk] - n[rj]) / s[rj]
        I = _t(tb.lagrange_time_integral(M, tau0, tau1))
        rjt, rlt, rkt = (torch.as_tensor(v, dtype=torch.long) for v in (rj, rl, rk))
        vbar = torch.einsum("rq,rqc->rc", I, vvel[rjt, rlt]) / _t(tau1 - tau0)[:, None]
        mu = Q[rjt, 0] * A[rjt]
        num = torch.zeros((self.NV, 2), dtype=_F64).index_add(0, rkt, mu[:, None] * vbar)
        den = torch.zeros(self.NV, dtype=_F64).index_add(0, rkt, mu)
        mt = torch.as_tensor(moved, dtype=torch.long)
        V = num[mt] / den[mt][:, None]
        wn = g.wall_n[mt]
        V = (V - (V * wn).sum(dim=1, keepdim=True) * wn) * g.wall_free[mt][:, None]
        dtk = _t((newtick[moved] - nk[moved]) * delta)
        return X.index_copy(0, mt, X[mt] + dtk[:, None] * V)

    def _patches(self, X, Xn, nk, newtick, swept, n, s, trace, avg, delta):
        """Fluxes G (E, 4), outward from L, over the swept edges' bilinear
        space-time patches; each side's predictor is read at its own rescaled
        time (tick - n) / s of the patch point."""
        M, cfg, topo = self.M, self.cfg, self.topo
        nG = M + 1
        chi, wc = tb.gauss_legendre01(nG)
        en = topo.edge_nodes
        a, b = en[swept, 0], en[swept, 1]
        L, R = topo.edge_elems[swept, 0], topo.edge_elems[swept, 1]
        el, er = topo.edge_local[swept, 0], topo.edge_local[swept, 1]
        hasR = R >= 0
        Rs = np.where(hasR, R, L)
        ers = np.where(hasR, er, el)
        if (s[L] <= 0).any() or (hasR & (s[Rs] <= 0)).any():
            raise AssertionError("patch neighbour without a valid predictor")
        ta, tbn = torch.as_tensor(a, dtype=torch.long), torch.as_tensor(b, dtype=torch.long)

        def col(v):
            return _t(v * delta)[:, None]

        P1 = torch.cat([X[ta], col(nk[a])], 1)
        P2 = torch.cat([X[tbn], col(nk[b])], 1)
        P3 = torch.cat([Xn[tbn], col(newtick[b])], 1)
        P4 = torch.cat([Xn[ta], col(newtick[a])], 1)
        ticks = np.stack([nk[a], nk[b], newtick[b], newtick[a]], 1).astype(float)
        lt_ = torch.as_tensor(L, dtype=torch.long)
        trL = trace[lt_, torch.as_tensor(el, dtype=torch.long)]
        trR = trace[torch.as_tensor(Rs, dtype=torch.long), torch.as_tensor(ers, dtype=torch.long)]
        avL = avg[lt_]
        slip_np = topo.bc_tag[swept] == BC_SLIP
        slip = torch.as_tensor(slip_np)
        open_ = torch.as_tensor(~hasR & ~slip_np)
        hasRt = torch.as_tensor(hasR)
        sRs = np.where(hasR, s[Rs], 1)
        G = torch.zeros((len(swept), 4), dtype=_F64)
        for gg in range(nG):
            for h in range(nG):
                c, t = float(chi[gg]), float(chi[h])
                dchi = (1 - t) * (P2 - P1) + t * (P3 - P4)
                dtau = (1 - c) * (P4 - P1) + c * (P3 - P2)
                N = torch.linalg.cross(dchi, dtau, dim=-1)
                tk = ((1 - c) * (1 - t) * ticks[:, 0] + c * (1 - t) * ticks[:, 1] + c * t * ticks[:, 2]
                      + (1 - c) * t * ticks[:, 3])
                lL = _t(tb.lagrange_time(M, (tk - n[L]) / s[L]))
                lR = _t(tb.lagrange_time(M, (tk - n[Rs]) / sRs))
                ql = torch.einsum("eq,eqv->ev", lL, trL[:, gg])
                qr = torch.where(slip[:, None], mirror(ql, N),
                                 torch.where(open_[:, None], torch.einsum("eq,eqv->ev", lL, avL), ql))
                qr = torch.where(hasRt[:, None], torch.einsum("eq,eqv->ev", lR, trR[:, nG - 1 - gg]), qr)
                G = G + (wc[gg] * wc[h]) * FLUX_FUNCTIONS[cfg.flux](ql, qr, N, cfg.gamma)
        return G, L, R, hasR

    # -- the macro step --------------------------------------------------------
    def macro(self, Q, X, W, delta, steps):
        """(Q', X', W') after one macro step of tick length delta from (Q, X, W)
        (torch: averages (NE, 4), positions (NV, 2), nodal reconstruction
        (NE, nb, 4) at the macro-step start); steps[i]: element i's steps."""
        from .scheme import MACRO_TICKS
        g, topo = self.g, self.topo
        NE, N = self.NE, MACRO_TICKS
        tris = topo.tris
        n = np.zeros(NE, np.int64)
        nk = np.zeros(self.NV, np.int64)
        pos = np.ones(NE, np.int64)
        s = np.array([st[0] for st in steps], np.int64)
        Xe = X[g.tris]
        A = _tri_area_t(Xe)
        trace, avg, vvel = g.predict(W, Xe, s * delta)
        QM = torch.zeros((NE, 4), dtype=_F64)
        en = topo.edge_nodes
        while (n < N).any():
            fut = n + s
            act = np.array([i for i in range(NE) if n[i] < N
                            and n[topo.sched[i]].max() <= fut[i] <= fut[topo.sched[i]].min()], np.int64)
            if act.size == 0:
                raise RuntimeError("deadlock: no element satisfies the update criterion")
            newtick = nk.copy()
            for i in act:
                for k in tris[i]:
                    if nk[k] < fut[i]:
                        newtick[k] = fut[i]
            moved = np.nonzero(newtick != nk)[0]
            Xn = self._move(X, Q, A, vvel, n, s, nk, newtick, moved, delta)
            is_moved = newtick != nk
            swept = np.nonzero(is_moved[en[:, 0]] | is_moved[en[:, 1]])[0]
            if swept.size:
                G, L, R, hasR = self._patches(X, Xn, nk, newtick, swept, n, s, trace, avg, delta)
                QM = QM.index_add(0, torch.as_tensor(L, dtype=torch.long), -G)
                QM = QM.index_add(0, torch.as_tensor(R[hasR], dtype=torch.long), G[torch.as_tensor(hasR)])
            X, nk = Xn, newtick
            ta = torch.as_tensor(act, dtype=torch.long)
            Xna = X[g.tris[ta]]
            An = _tri_area_t(Xna)
            Q = Q.index_copy(0, ta, (A[ta, None] * Q[ta] + QM[ta]) / An[:, None])
            QM = QM.index_copy(0, ta, torch.zeros((act.size, 4), dtype=_F64))
            A = A.index_copy(0, ta, An)
            Xe = Xe.index_copy(0, ta, Xna)
            n[act] = fut[act]
            W = W.index_copy(0, ta, self._reconstruct(act, Q, Xe, avg, vvel, n, s, delta))
            going = act[n[act] < N]
            s[act[n[act] >= N]] = 0
            for i in going:
                s[i] = steps[i][pos[i]]
                pos[i] += 1
            if going.size:
                tg = torch.as_tensor(going, dtype=torch.long)
                tr, av, vv = g.predict(W[tg], Xe[tg], s[going] * delta)
                trace = trace.index_copy(0, tg, tr)
                avg = avg.index_copy(0, tg, av)
                vvel = vvel.index_copy(0, tg, vv)
        if any(pos[i] != len(steps[i]) for i in range(NE)):
            raise ValueError("the schedule does not match the macro step")
        return Q, X, W

    def initial(self, Q, X):
        """The reconstruction of the pre-processing (real neighbours)."""
        return self.g.reconstruct(Q, X[self.g.tris])

    def run(self, Q0, X0, schedule):
        """(Q, X) after the macro steps of `schedule` from (Q0, X0), NumPy in and out."""
        with torch.no_grad():
            Q, X = _t(Q0), _t(X0)
            W = self.initial(Q, X)
            for delta, steps in schedule:
                Q, X, W = self.macro(Q, X, W, delta, steps)
        return Q.numpy(), X.numpy()

    def vjp(self, Q0, X0, schedule, Qbar, Xbar):
        """Adjoints of (Q0, X0) (through the pre-processing reconstruction too)
        for the adjoints (Qbar, Xbar) of the final (Q, X); NumPy in and out."""
        q = _t(Q0).requires_grad_(True)
        x = _t(X0).requires_grad_(True)
        Q, X, W = q, x, self.initial(q, x)
        for delta, steps in schedule:
            Q, X, W = self.macro(Q, X, W, delta, steps)
        gq, gx = torch.autograd.grad((Q, X), (q, x), (_t(Qbar), _t(Xbar)))
        return gq.detach().numpy(), gx.detach().numpy()
