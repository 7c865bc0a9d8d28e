"""Invariants of the oracle's topology and stencils (paper Sec. 2.2: stencils of
n_e = 2*nb elements, 1 central + 3 primary + 3 reverse sector stencils, and a
symmetric total stencil for the update criterion)."""
import numpy as np
import pytest

from oracle.topology import barycentres, build_topology
from workloads import square_graded_mesh, strip_mesh


@pytest.fixture(scope="module", params=[1, 2, 3])
def topo_case(request):
    mesh = square_graded_mesh(0.35, seed=9)
    return mesh, request.param, build_topology(mesh.nodes, mesh.tris, request.param)


def test_edges_and_neighbours(topo_case):
    mesh, M, t = topo_case
    NE = mesh.n_elems
    # Euler characteristic of a disk-like triangulation: V - E + F = 1
    assert mesh.n_nodes - t.edge_nodes.shape[0] + NE == 1
    for e in range(t.edge_nodes.shape[0]):
        a, b = t.edge_nodes[e]
        L, R = t.edge_elems[e]
        kl = t.edge_local[e, 0]
        assert (t.tris[L, kl], t.tris[L, (kl + 1) % 3]) == (a, b)
        if R >= 0:
            kr = t.edge_local[e, 1]
            assert (t.tris[R, kr], t.tris[R, (kr + 1) % 3]) == (b, a)
            assert t.neigh[L, kl] == R and t.neigh[R, kr] == L
    assert (t.bc_tag[t.edge_elems[:, 1] < 0] > 0).all()


def test_stencil_shapes(topo_case):
    mesh, M, t = topo_case
    ne = (M + 1) * (M + 2)
    bc = barycentres(mesh.nodes, mesh.tris)
    for i in range(mesh.n_elems):
        for s in range(7):
            st = t.stencils[i, s]
            if st[0] < 0:
                assert s > 0 and (st < 0).all()
                continue
            assert st[0] == i and len(set(st.tolist())) == ne
            if s == 0:
                # face neighbours come first in the central stencil
                nb = set(t.neigh[i][t.neigh[i] >= 0].tolist())
                assert nb <= set(st[1:1 + len(nb)].tolist())
            else:
                k = (s - 1) % 3
                X = mesh.nodes[mesh.tris[i]]
                P, e1, e2 = X[k], X[(k + 1) % 3] - X[k], X[(k + 2) % 3] - X[k]
                d = bc[st[1:]] - P
                c1 = d[:, 0] * e2[1] - d[:, 1] * e2[0]
                c2 = e1[0] * d[:, 1] - e1[1] * d[:, 0]
                sign = 1 if s <= 3 else -1
                assert (sign * c1 > 0).all() and (sign * c2 > 0).all()
    # interior elements keep most sector stencils
    assert (t.stencils[:, :, 0] >= 0).sum() > 4.5 * mesh.n_elems


def test_scheduling_stencil_symmetric(topo_case):
    mesh, M, t = topo_case
    member = [set(s.tolist()) for s in t.sched]
    for i in range(mesh.n_elems):
        assert i in member[i]
        for j in member[i]:
            assert i in member[j]
        st = t.stencils[i][t.stencils[i, :, 0] >= 0].ravel()
        assert set(st.tolist()) <= member[i]
    for k in range(mesh.n_nodes):
        ring = [r[0] for r in t.ring[k]]
        for i in ring:
            assert set(ring) <= member[i]


def test_inconsistent_orientation_rejected():
    mesh = strip_mesh(0, 1, 0, 1, 0.3, seed=1)
    tris = mesh.tris.copy()
    tris[0] = tris[0, [0, 2, 1]]
    with pytest.raises(ValueError):
        build_topology(mesh.nodes, tris, 1)
