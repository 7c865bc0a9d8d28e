"""Mesh topology and reconstruction stencils (oracle, test infrastructure).

Definitions (the paper defers the stencil algorithm to its references, Sec. 2.2
around eqs. stencil and eqn.WENOstencil; the readings below are the ones this
code implements, stated so that an independent implementation can match them):

  * Edges are numbered in order of first appearance when the elements are
    walked in index order with local edges k = 0,1,2 (local edge k runs from
    local vertex k to k+1).  The first element is the edge's left element L and
    the edge is oriented as in L; the other element, if any, is R.
  * Barycentre c_j = ((x1+x2+x3)/3, (y1+y2+y3)/3); distance key d2 = dx*dx + dy*dy.
  * Stencil size n_e = 2 * nb elements, element i first (eq. stencil).
  * Central stencil: breadth-first layers over face neighbours; elements taken
    by (layer, d2, index) until n_e are collected.
  * Sector stencils at local vertex k (apex P = X_k, e1 = X_{k+1}-P, e2 = X_{k+2}-P,
    d = c_j - P): primary sector admits c_j with cross(d,e2) > 0 and
    cross(e1,d) > 0 (the cone spanned by e1, e2); reverse sector admits
    cross(d,e2) < 0 and cross(e1,d) < 0 (the cone spanned by -e1, -e2).
    Candidates are the elements at vertex-adjacency distance 1..M+4 from i;
    the admitted ones are ranked by (d2, index) and the first n_e - 1 follow i.
    A sector with fewer admitted candidates is dropped (marked -1).
    Stencil order: s=0 central, s=1..3 primary at vertices 0..2, s=4..6 reverse.
  * Scheduling stencil: U_i = (union of the 7 stencils) + (all elements sharing
    a node with i); S_i = { j : j in U_i or i in U_j }, the symmetric closure
    required for deadlock freedom (discussion after eq. eqn.WENOupdate).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from .tables import sizes


@dataclasses.dataclass
class Topology:
    n_nodes: int
    n_elems: int
    tris: np.ndarray          # (NE,3)
    edge_nodes: np.ndarray    # (NF,2) a,b oriented as in L
    edge_elems: np.ndarray    # (NF,2) L, R (R=-1 boundary)
    edge_local: np.ndarray    # (NF,2) local edge index in L, in R (-1)
    elem_edges: np.ndarray    # (NE,3) edge id of local edge k
    neigh: np.ndarray         # (NE,3) element across local edge k or -1
    ring: list                # per node: list of (elem, local vertex) by elem index
    stencils: np.ndarray      # (NE,7,ne) int, -1 rows for dropped stencils
    sched: list               # per element: sorted array of the scheduling stencil
    bc_tag: np.ndarray        # (NF,) boundary tag (0 interior)


def build_edges(tris: np.ndarray):
    ne_ = tris.shape[0]
    key_to_edge = {}
    edge_nodes, edge_elems, edge_local = [], [], []
    elem_edges = np.zeros((ne_, 3), np.int64)
    for i in range(ne_):
        for k in range(3):
            a, b = int(tris[i, k]), int(tris[i, (k + 1) % 3])
            key = (min(a, b), max(a, b))
            e = key_to_edge.get(key)
            if e is None:
                e = len(edge_nodes)
                key_to_edge[key] = e
                edge_nodes.append([a, b])
                edge_elems.append([i, -1])
                edge_local.append([k, -1])
            else:
                if edge_elems[e][1] != -1 or edge_nodes[e] != [b, a]:
                    raise ValueError("mesh is not a consistently oriented manifold")
                edge_elems[e][1] = i
                edge_local[e][1] = k
            elem_edges[i, k] = e
    return (np.array(edge_nodes, np.int64), np.array(edge_elems, np.int64),
            np.array(edge_local, np.int64), elem_edges)


def barycentres(nodes, tris):
    p = nodes[tris]
    return np.stack([(p[:, 0, 0] + p[:, 1, 0] + p[:, 2, 0]) / 3.0,
                     (p[:, 0, 1] + p[:, 1, 1] + p[:, 2, 1]) / 3.0], axis=1)


def _central(i, neigh, bc, ne):
    seen = {i}
    out = [i]
    layer = [i]
    while len(out) < ne and layer:
        nxt = []
        for j in layer:
            for k in range(3):
                m = int(neigh[j, k])
                if m >= 0 and m not in seen:
                    seen.add(m)
                    nxt.append(m)
        dx = bc[nxt, 0] - bc[i, 0] if nxt else np.zeros(0)
        dy = bc[nxt, 1] - bc[i, 1] if nxt else np.zeros(0)
        d2 = dx * dx + dy * dy
        order = sorted(range(len(nxt)), key=lambda t: (d2[t], nxt[t]))
        for t in order:
            if len(out) < ne:
                out.append(nxt[t])
        layer = nxt
    if len(out) < ne:
        raise ValueError(f"mesh too small: central stencil of element {i} has {len(out)} < {ne}")
    return out


def _vertex_reach(tris, NV, M):
    """Vertex adjacency of the elements and the candidate pools within M+4
    vertex layers (sparse, sorted indices)."""
    NE = tris.shape[0]
    rows = np.repeat(np.arange(NE), 3)
    en = sp.csr_matrix((np.ones(3 * NE), (rows, tris.ravel())), shape=(NE, NV))
    adj = (en @ en.T).tocsr()
    adj.data[:] = 1.0
    reach = adj.copy()
    for _ in range(M + 3):
        reach = (reach @ adj).tocsr()
        reach.data[:] = 1.0
    reach.sort_indices()
    return adj, reach


def _element_stencils(i, nodes, tris, neigh, bc, reach, ne):
    """The 7 stencils of element i (eqs. stencil, eqn.WENOstencil): central
    (face-neighbour layers), then for each vertex the primary and the reverse
    sector; a sector without ne - 1 candidates stays -1."""
    out = -np.ones((7, ne), np.int64)
    out[0] = _central(i, neigh, bc, ne)
    cand = reach.indices[reach.indptr[i]:reach.indptr[i + 1]]
    cand = cand[cand != i]
    dxc = bc[cand, 0] - bc[i, 0]
    dyc = bc[cand, 1] - bc[i, 1]
    d2 = dxc * dxc + dyc * dyc
    X = nodes[tris[i]]
    for k in range(3):
        P = X[k]
        e1 = X[(k + 1) % 3] - P
        e2 = X[(k + 2) % 3] - P
        dx = bc[cand, 0] - P[0]
        dy = bc[cand, 1] - P[1]
        c1 = dx * e2[1] - dy * e2[0]        # cross(d, e2)
        c2 = e1[0] * dy - e1[1] * dx        # cross(e1, d)
        for s, mask in ((1 + k, (c1 > 0) & (c2 > 0)), (4 + k, (c1 < 0) & (c2 < 0))):
            idx = np.nonzero(mask)[0]
            if idx.size < ne - 1:
                continue
            order = np.lexsort((cand[idx], d2[idx]))[: ne - 1]
            out[s, 0] = i
            out[s, 1:] = cand[idx][order]
    return out


def face_neighbours(tris: np.ndarray) -> np.ndarray:
    """(NE, 3) element across local edge k, -1 on the boundary."""
    tris = np.asarray(tris, np.int64)
    edge_nodes, edge_elems, edge_local, _ = build_edges(tris)
    neigh = -np.ones((tris.shape[0], 3), np.int64)
    inner = edge_elems[:, 1] >= 0
    L, R = edge_elems[inner, 0], edge_elems[inner, 1]
    neigh[L, edge_local[inner, 0]] = R
    neigh[R, edge_local[inner, 1]] = L
    return neigh


def stencils_of(nodes: np.ndarray, tris: np.ndarray, M: int, elems) -> np.ndarray:
    """The 7 stencils of the given elements only (same construction as
    build_topology), for sampled checks on meshes too large to process whole."""
    nodes = np.asarray(nodes, float)
    tris = np.asarray(tris, np.int64)
    ne = sizes(M)["ne"]
    neigh = face_neighbours(tris)
    bc = barycentres(nodes, tris)
    _, reach = _vertex_reach(tris, nodes.shape[0], M)
    return np.stack([_element_stencils(int(i), nodes, tris, neigh, bc, reach, ne) for i in elems])


def build_topology(nodes: np.ndarray, tris: np.ndarray, M: int, bedges=None) -> Topology:
    nodes = np.asarray(nodes, float)
    tris = np.asarray(tris, np.int64)
    NE, NV = tris.shape[0], nodes.shape[0]
    ne = sizes(M)["ne"]
    edge_nodes, edge_elems, edge_local, elem_edges = build_edges(tris)
    neigh = -np.ones((NE, 3), np.int64)
    for e in range(edge_nodes.shape[0]):
        L, R = edge_elems[e]
        if R >= 0:
            neigh[L, edge_local[e, 0]] = R
            neigh[R, edge_local[e, 1]] = L
    bc_tag = np.zeros(edge_nodes.shape[0], np.int64)
    bmask = edge_elems[:, 1] < 0
    bc_tag[bmask] = 1
    if bedges is not None:
        tag = {(int(a), int(b)): int(t) for a, b, t in np.asarray(bedges)}
        for e in np.nonzero(bmask)[0]:
            a, b = edge_nodes[e]
            if (int(a), int(b)) not in tag:
                raise ValueError("boundary edge list does not match the mesh boundary")
            bc_tag[e] = tag[(int(a), int(b))]
    ring = [[] for _ in range(NV)]
    for i in range(NE):
        for k in range(3):
            ring[int(tris[i, k])].append((i, k))
    bc = barycentres(nodes, tris)
    adj, reach = _vertex_reach(tris, NV, M)
    stencils = -np.ones((NE, 7, ne), np.int64)
    for i in range(NE):
        stencils[i] = _element_stencils(i, nodes, tris, neigh, bc, reach, ne)

    # scheduling stencil: symmetric closure of stencils + vertex ring
    U = [set() for _ in range(NE)]
    for i in range(NE):
        st = stencils[i][stencils[i, :, 0] >= 0].ravel()
        U[i].update(int(j) for j in st)
        U[i].update(int(j) for j in adj.indices[adj.indptr[i]:adj.indptr[i + 1]])
        U[i].add(i)
    S = [set(u) for u in U]
    for i in range(NE):
        for j in U[i]:
            S[j].add(i)
    sched = [np.array(sorted(s), np.int64) for s in S]
    return Topology(NV, NE, tris, edge_nodes, edge_elems, edge_local, elem_edges, neigh,
                    ring, stencils, sched, bc_tag)
