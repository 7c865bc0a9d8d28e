"""Seeded triangular meshes for the synthetic workloads.

Point sets are built from a jittered hexagonal lattice (uniform size) or from
jittered concentric rings (radially graded size), triangulated with
``scipy.spatial.Delaunay``, oriented counter-clockwise and renumbered along a
Hilbert curve so that neighbouring triangles and nodes sit close in memory.

Every domain used here is convex, so the convex hull edges are the boundary
edges.  All boundary edges carry tag 1 (transmissive).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.spatial import Delaunay

BC_TRANSMISSIVE = 1
BC_SLIP = 2


@dataclasses.dataclass
class Mesh:
    nodes: np.ndarray   # (NV, 2) float64
    tris: np.ndarray    # (NE, 3) int32, counter-clockwise
    bedges: np.ndarray  # (NB, 3) int32: node a, node b, tag; interior lies left of a->b
    name: str = ""

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.tris.shape[0])

    def areas(self) -> np.ndarray:
        p = self.nodes[self.tris]
        return 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                      - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))


# ---------------------------------------------------------------------------
# Hilbert ordering
# ---------------------------------------------------------------------------
def _hilbert_index(ix: np.ndarray, iy: np.ndarray, order: int) -> np.ndarray:
    """Hilbert-curve index of integer cell coordinates on a 2^order grid."""
    x = ix.astype(np.int64).copy()
    y = iy.astype(np.int64).copy()
    d = np.zeros_like(x)
    s = 1 << (order - 1)
    while s > 0:
        rx = ((x & s) > 0).astype(np.int64)
        ry = ((y & s) > 0).astype(np.int64)
        d += s * s * ((3 * rx) ^ ry)
        # rotate the quadrant
        flip = ry == 0
        swap_x = np.where(flip & (rx == 1), s - 1 - x, x)
        swap_y = np.where(flip & (rx == 1), s - 1 - y, y)
        x = np.where(flip, swap_y, swap_x)
        y = np.where(flip, swap_x, swap_y)
        s >>= 1
    return d


def _hilbert_order(points: np.ndarray, order: int = 16) -> np.ndarray:
    lo = points.min(axis=0)
    span = max(float((points.max(axis=0) - lo).max()), 1e-300)
    g = np.clip(((points - lo) / span * ((1 << order) - 1)).astype(np.int64), 0, (1 << order) - 1)
    return np.argsort(_hilbert_index(g[:, 0], g[:, 1], order), kind="stable")


# ---------------------------------------------------------------------------
# Triangulation and clean-up
# ---------------------------------------------------------------------------
def _triangulate(points: np.ndarray, name: str) -> Mesh:
    tri = Delaunay(points)
    tris = tri.simplices.astype(np.int64)
    p = points[tris]
    area2 = ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
             - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    neg = area2 < 0
    tris[neg] = tris[neg][:, [0, 2, 1]]
    area2 = np.abs(area2)
    # drop hull slivers made of (nearly) collinear boundary points
    scale = np.median(area2)
    keep = area2 > 1e-9 * scale
    tris = tris[keep]
    used = np.zeros(points.shape[0], bool)
    used[tris.ravel()] = True
    # renumber nodes along a Hilbert curve (unused points dropped)
    node_order = [i for i in _hilbert_order(points) if used[i]]
    node_order = np.asarray(node_order, np.int64)
    remap = -np.ones(points.shape[0], np.int64)
    remap[node_order] = np.arange(node_order.size)
    nodes = points[node_order].copy()
    tris = remap[tris]
    cent = nodes[tris].mean(axis=1)
    tris = tris[_hilbert_order(cent)]
    # rotate each triangle so that its smallest node index comes first (canonical form)
    rot = np.argmin(tris, axis=1)
    tris = np.stack([tris[np.arange(len(tris)), (rot + k) % 3] for k in range(3)], axis=1)
    bedges = _boundary_edges(tris)
    return Mesh(nodes=nodes, tris=tris.astype(np.int32), bedges=bedges, name=name)


def _boundary_edges(tris: np.ndarray) -> np.ndarray:
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    key = np.sort(e, axis=1)
    _, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    inv = inv.ravel()
    if cnt.max() > 2:
        raise ValueError("non-manifold triangulation")
    b = e[cnt[inv] == 1]
    out = np.empty((b.shape[0], 3), np.int32)
    out[:, 0:2] = b
    out[:, 2] = BC_TRANSMISSIVE
    return out


# ---------------------------------------------------------------------------
# Point sets
# ---------------------------------------------------------------------------
def _disk_jitter(rng, n, radius):
    r = radius * np.sqrt(rng.random(n))
    a = 2 * math.pi * rng.random(n)
    return np.stack([r * np.cos(a), r * np.sin(a)], axis=1)


def strip_mesh(x0: float, x1: float, y0: float, y1: float, h: float, seed: int,
               name: str = "strip", slip_y: bool = False) -> Mesh:
    """Uniform mesh of a rectangle: jittered hexagonal lattice (jitter <= 0.25 h).
    With slip_y the sides y = y0 and y = y1 are slip walls (tag 2), the others
    transmissive (tag 1)."""
    rng = np.random.default_rng(seed)
    ny = max(2, int(round((y1 - y0) / (h * math.sqrt(3) / 2))))
    dy = (y1 - y0) / ny
    nx = max(2, int(round((x1 - x0) / h)))
    dx = (x1 - x0) / nx
    pts = []
    for j in range(1, ny):
        off = 0.5 * dx if j % 2 else 0.0
        xs = x0 + off + dx * np.arange(nx + 1)
        xs = xs[(xs > x0 + 0.45 * dx) & (xs < x1 - 0.45 * dx)]
        pts.append(np.stack([xs, np.full_like(xs, y0 + j * dy)], axis=1))
    inner = np.concatenate(pts)
    inner = inner + _disk_jitter(rng, inner.shape[0], 0.25 * min(dx, dy))
    bx = x0 + dx * np.arange(nx + 1)
    by = y0 + dy * np.arange(1, ny)
    bnd = np.concatenate([
        np.stack([bx, np.full_like(bx, y0)], 1), np.stack([bx, np.full_like(bx, y1)], 1),
        np.stack([np.full_like(by, x0), by], 1), np.stack([np.full_like(by, x1), by], 1)])
    mesh = _triangulate(np.concatenate([bnd, inner]), name)
    if slip_y:
        ya = mesh.nodes[mesh.bedges[:, 0], 1]
        yb = mesh.nodes[mesh.bedges[:, 1], 1]
        wall = ((ya == y0) & (yb == y0)) | ((ya == y1) & (yb == y1))
        mesh.bedges[wall, 2] = BC_SLIP
    return mesh


def _ring_radii(hfun, r_max: float, exact_end: bool):
    radii = [0.0]
    r = 0.0
    while r < r_max:
        dr = 0.866 * hfun(r + 0.433 * hfun(r))
        r = r + dr
        radii.append(r)
    radii = np.asarray(radii)
    if exact_end:
        # close the last ring exactly on r_max
        if radii[-1] - r_max > 0.5 * (radii[-1] - radii[-2]):
            radii = radii[:-1]
        radii = radii * (r_max / radii[-1])
    return radii


def _ring_points(rng, center, radii, hfun, jitter, last_exact):
    pts = [np.asarray(center, float)[None, :]]
    for k, r in enumerate(radii[1:], start=1):
        h = hfun(r)
        n = max(6, int(round(2 * math.pi * r / h)))
        a = 2 * math.pi * (np.arange(n) + rng.random()) / n
        rr = np.full(n, r)
        if not (last_exact and k == len(radii) - 1):
            a = a + jitter * (rng.random(n) - 0.5) * 2 * h / r
            rr = rr + jitter * (rng.random(n) - 0.5) * 2 * h
        pts.append(np.stack([center[0] + rr * np.cos(a), center[1] + rr * np.sin(a)], 1))
    return np.concatenate(pts)


def disk_graded_mesh(h_min: float, seed: int, grading: float = 8.0, r_fine: float = 0.5,
                     radius: float = 1.0, name: str = "disk") -> Mesh:
    """Unit disk with a radial size function, finest at r = r_fine and `grading`
    times coarser at the centre and the rim (jittered concentric rings)."""
    rng = np.random.default_rng(seed)

    def hfun(r):
        return h_min * min(grading, 1.0 + (grading - 1.0) * abs(r - r_fine) / r_fine)

    radii = _ring_radii(hfun, radius, exact_end=True)
    pts = _ring_points(rng, (0.0, 0.0), radii, hfun, 0.12, last_exact=True)
    return _triangulate(pts, name)


def square_graded_mesh(h_fine: float, seed: int, lo: float = 0.0, hi: float = 10.0,
                       r1: float = 1.5, r2: float = 3.5, ratio: float = 4.0,
                       name: str = "square") -> Mesh:
    """Square [lo,hi]^2 with size h_fine for r < r1 around the centre, growing
    linearly to ratio*h_fine at r >= r2 (jittered rings clipped to the square)."""
    rng = np.random.default_rng(seed)
    c = 0.5 * (lo + hi)

    def hfun(r):
        if r <= r1:
            return h_fine
        if r >= r2:
            return ratio * h_fine
        return h_fine * (1.0 + (ratio - 1.0) * (r - r1) / (r2 - r1))

    radii = _ring_radii(hfun, math.sqrt(2) * (hi - c) + 2 * ratio * h_fine, exact_end=False)
    pts = _ring_points(rng, (c, c), radii, hfun, 0.12, last_exact=False)
    r_of = np.hypot(pts[:, 0] - c, pts[:, 1] - c)
    hloc = np.array([hfun(r) for r in r_of])
    dist = np.minimum.reduce([pts[:, 0] - lo, hi - pts[:, 0], pts[:, 1] - lo, hi - pts[:, 1]])
    pts = pts[dist > 0.6 * hloc]
    # boundary points, marching along each side with the local size; the
    # marched positions are stretched so the last one lands on the corner
    bnd = []
    side = hi - lo

    def on_side(k, s):
        return [(lo + s, lo), (hi, lo + s), (hi - s, hi), (lo, hi - s)][k]

    for k in range(4):
        svals = [0.0]
        while svals[-1] < side:
            p = on_side(k, svals[-1])
            svals.append(svals[-1] + hfun(math.hypot(p[0] - c, p[1] - c)))
        if len(svals) > 2 and svals[-1] - side > 0.5 * (svals[-1] - svals[-2]):
            svals = svals[:-1]
        svals = np.asarray(svals) * (side / svals[-1])
        for s in svals[:-1]:
            bnd.append(on_side(k, s))
    bnd = np.asarray(bnd)
    return _triangulate(np.concatenate([bnd, pts]), name)
