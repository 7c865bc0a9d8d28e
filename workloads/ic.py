"""Initial conditions and their cell averages for the synthetic workloads.

Primitive states follow the paper's test section: the Sod data of the Riemann
problem table (RP1), the EP1 row of the explosion table, and the isentropic
vortex of the convergence study (eqs. ShuVortIC, ShuVortDelta, rhopressDelta).
Cell averages are taken with a collapsed (Duffy) 8x8 Gauss rule per triangle;
they are inputs handed to both the GPU path and the oracle.
"""
from __future__ import annotations

import math

import numpy as np

from .mesh import Mesh, strip_mesh, square_graded_mesh, disk_graded_mesh


def _gauss01(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _duffy(n: int):
    u, wu = _gauss01(n)
    U, V = np.meshgrid(u, u, indexing="ij")
    WU, WV = np.meshgrid(wu, wu, indexing="ij")
    xi = (U * (1 - V)).ravel()
    eta = V.ravel()
    w = (WU * WV * (1 - V)).ravel()
    return xi, eta, w / w.sum()


def prim_to_cons(prim: np.ndarray, gamma: float) -> np.ndarray:
    rho, u, v, p = prim[..., 0], prim[..., 1], prim[..., 2], prim[..., 3]
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1) + 0.5 * rho * (u * u + v * v)], -1)


def cell_average(mesh: Mesh, prim_fn, gamma: float, n: int = 8) -> np.ndarray:
    """Average of the conserved initial state over every triangle, (NE, 4)."""
    xi, eta, w = _duffy(n)
    p = mesh.nodes[mesh.tris]                      # (NE, 3, 2)
    x = (p[:, None, 0, :] + (p[:, None, 1, :] - p[:, None, 0, :]) * xi[None, :, None]
         + (p[:, None, 2, :] - p[:, None, 0, :]) * eta[None, :, None])
    q = prim_to_cons(prim_fn(x[..., 0], x[..., 1]), gamma)
    return np.einsum("eqv,q->ev", q, w)


def sod_primitive(x, y, left=(1.0, 0.0, 0.0, 1.0), right=(0.125, 0.0, 0.0, 0.1), xd=0.0):
    out = np.empty(np.shape(x) + (4,))
    lm = np.asarray(x) < xd
    out[lm] = left
    out[~lm] = right
    return out


def explosion_primitive(x, y, inner=(1.0, 0.0, 0.0, 1.0), outer=(0.125, 0.0, 0.0, 0.1), r0=0.5):
    out = np.empty(np.shape(x) + (4,))
    im = np.hypot(x, y) < r0
    out[im] = inner
    out[~im] = outer
    return out


def vortex_primitive(x, y, eps=5.0, gamma=1.4, xc=5.0, yc=5.0):
    dx, dy = x - xc, y - yc
    r2 = dx * dx + dy * dy
    amp = eps / (2 * math.pi) * np.exp(0.5 * (1 - r2))
    dT = -(gamma - 1) * eps * eps / (8 * gamma * math.pi ** 2) * np.exp(1 - r2)
    rho = (1 + dT) ** (1 / (gamma - 1))
    p = (1 + dT) ** (gamma / (gamma - 1))
    return np.stack([rho, 1 - amp * dy, 1 + amp * dx, p], -1)


# ---------------------------------------------------------------------------
# Named cases
# ---------------------------------------------------------------------------
def _calibrated(make, h0: float, target: int, iters: int = 3) -> Mesh:
    h = h0
    mesh = make(h)
    for _ in range(iters):
        if abs(mesh.n_elems - target) <= 0.01 * target:
            break
        h *= math.sqrt(mesh.n_elems / target)
        mesh = make(h)
    return mesh


def sod_case(n_target: int = 2000, seed: int = 1408, gamma: float = 1.4):
    """Sod tube on [-0.5,0.5]x[0,0.1] (paper RP1 data; strip height per the
    shock-tube workload), uniform jittered mesh, slip walls at y = 0 and 0.1
    and transmissive ends."""
    mesh = _calibrated(lambda h: strip_mesh(-0.5, 0.5, 0.0, 0.1, h, seed, "sod", slip_y=True),
                       0.0107, n_target)
    return mesh, cell_average(mesh, sod_primitive, gamma)


def vortex_case(n_target: int = 5000, seed: int = 1, gamma: float = 1.4):
    """Isentropic vortex (strength 5) on [0,10]^2 with a 4:1 graded mesh."""
    mesh = _calibrated(lambda h: square_graded_mesh(h, seed, name="vortex"),
                       math.sqrt(43.0 / n_target), n_target)
    return mesh, cell_average(mesh, lambda x, y: vortex_primitive(x, y, gamma=gamma), gamma)


def explosion_case(n_target: int = 400_000, seed: int = 7, gamma: float = 1.4,
                   inner=(1.0, 0.0, 0.0, 1.0), outer=(0.125, 0.0, 0.0, 0.1)):
    """EP1 explosion on the unit disk, 8:1 radially graded mesh finest at r=0.5."""
    mesh = _calibrated(lambda h: disk_graded_mesh(h, seed, name="explosion"),
                       math.sqrt(1.2 / n_target), n_target)
    return mesh, cell_average(mesh, lambda x, y: explosion_primitive(x, y, inner, outer), gamma)


def batched_cases(n_instances: int = 256, seed: int = 256, n_min: int = 1000,
                  n_max: int = 50_000, gamma: float = 1.4):
    """Uneven batch of Riemann (even index) and explosion (odd index) instances
    with log-uniform sizes and random left/right density and pressure."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_instances):
        n = int(round(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        rl, rr, pl, pr = rng.uniform(0.1, 2.0, 4)
        if k % 2 == 0:
            mesh = strip_mesh(-0.5, 0.5, 0.0, 0.1, math.sqrt(0.1 * 2.3 / n), seed + k, "tube",
                              slip_y=True)
            q = cell_average(mesh, lambda x, y: sod_primitive(
                x, y, (rl, 0, 0, pl), (rr, 0, 0, pr)), gamma)
        else:
            mesh = disk_graded_mesh(math.sqrt(1.2 / n), seed + k, name="disk")
            q = cell_average(mesh, lambda x, y: explosion_primitive(
                x, y, (rl, 0, 0, pl), (rr, 0, 0, pr)), gamma)
        out.append((mesh, q))
    return out


def concat_instances(cases):
    """Concatenate independent (mesh, Q) instances into one disjoint mesh.
    Returns nodes, tris, bedges, Q and elem_first: instance k owns elements
    elem_first[k]:elem_first[k+1] and the nodes of those elements."""
    nodes, tris, bedges, qs, first = [], [], [], [], [0]
    off = 0
    for mesh, q in cases:
        nodes.append(mesh.nodes)
        tris.append(mesh.tris + off)
        b = mesh.bedges.copy()
        b[:, :2] += off
        bedges.append(b)
        qs.append(q)
        off += mesh.nodes.shape[0]
        first.append(first[-1] + mesh.tris.shape[0])
    return (np.concatenate(nodes), np.concatenate(tris).astype(np.int32),
            np.concatenate(bedges).astype(np.int32), np.concatenate(qs),
            np.array(first, np.int32))
