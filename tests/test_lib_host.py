"""CPU-only checks of the native library: it loads, exports every symbol of
include/aderweno.h, and its host-side topology and tables (built
independently in C++) agree with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import tables as tb
from oracle.topology import build_topology
from paper_1408_3719_amd import Config, HostTopology, _lib
from workloads import square_graded_mesh, strip_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    header = open(os.path.join(ROOT, "include", "aderweno.h")).read()
    declared = set(re.findall(r"\b(ader_[a-z_]+)\s*\(", header))
    assert declared == set(_lib.EXPORTED)
    for name in declared:
        assert hasattr(lib, name), name


def test_invalid_configuration_rejected():
    lib = _lib.load()
    ctx = ctypes.c_void_p()
    for bad in (Config(M=4), Config(cfl=0.0), Config(levels=9), Config(weno_r=6.0)):
        c = bad.to_c()
        assert lib.ader_create(ctypes.byref(c), None, ctypes.byref(ctx)) == -1


def test_flux_selection():
    """Rusanov, Osher and HLL are accepted; other flux codes are rejected."""
    lib = _lib.load()
    for name in ("rusanov", "osher", "hll"):
        ctx = ctypes.c_void_p()
        c = Config(flux=name).to_c()
        assert lib.ader_create(ctypes.byref(c), None, ctypes.byref(ctx)) == 0
        lib.ader_destroy(ctx)
    ctx = ctypes.c_void_p()
    c = Config().to_c()
    c.flux = 3
    assert lib.ader_create(ctypes.byref(c), None, ctypes.byref(ctx)) == -1


def test_instance_ranges_validated():
    """ader_set_instances: contiguous element ranges over disjoint meshes only."""
    from workloads import concat_instances, sod_case, vortex_case
    nodes, tris, bedges, _, first = concat_instances([sod_case(300, seed=2), vortex_case(400, seed=3)])
    host = HostTopology(nodes, tris, bedges, Config(M=2))
    lib = host.lib
    f = np.ascontiguousarray(first, np.int32)
    assert lib.ader_set_instances(host.ctx, 2, f.ctypes.data) == 0
    bad = f.copy()
    bad[1] = bad[1] + 5                  # splits a mesh: the two ranges share nodes
    assert lib.ader_set_instances(host.ctx, 2, bad.ctypes.data) == -2
    bad = f.copy()
    bad[2] -= 1                          # does not end at n_elems
    assert lib.ader_set_instances(host.ctx, 2, bad.ctypes.data) == -1
    one = np.array([0, tris.shape[0]], np.int32)
    assert lib.ader_set_instances(host.ctx, 1, one.ctypes.data) == 0


def test_mesh_errors():
    mesh = strip_mesh(0, 1, 0, 1, 0.2, seed=1)
    tris = mesh.tris.copy()
    tris[0] = tris[0, [0, 2, 1]]
    with pytest.raises(_lib.AderError, match="E_MESH"):
        HostTopology(mesh.nodes, tris, mesh.bedges, Config(M=1))
    with pytest.raises(_lib.AderError, match="E_MESH"):
        HostTopology(mesh.nodes, mesh.tris, mesh.bedges[1:], Config(M=1))


@pytest.fixture(scope="module", params=[1, 2, 3])
def both(request):
    M = request.param
    mesh = square_graded_mesh(0.3, seed=3) if M < 3 else square_graded_mesh(0.25, seed=3)
    host = HostTopology(mesh.nodes, mesh.tris, mesh.bedges, Config(M=M))
    ora = build_topology(mesh.nodes, mesh.tris, M, mesh.bedges)
    return M, mesh, host, ora


def test_threaded_topology_matches_oracle():
    """Above 4096 elements the host builds stencils on several threads: the
    result is still the oracle's, bit for bit (two disjoint instances)."""
    from workloads import concat_instances, vortex_case
    nodes, tris, bedges, _, _ = concat_instances([vortex_case(3000, seed=4), vortex_case(2500, seed=6)])
    host = HostTopology(nodes, tris, bedges, Config(M=2))
    ora = build_topology(nodes, tris, 2, bedges)
    assert tris.shape[0] > 4096
    assert np.array_equal(host.dump("TOPO_STENCILS"), ora.stencils)
    ptr, idx = host.dump("TOPO_SCHED_PTR"), host.dump("TOPO_SCHED_IDX")
    for i in range(tris.shape[0]):
        assert np.array_equal(idx[ptr[i]:ptr[i + 1]], ora.sched[i]), i


def test_edges_match_oracle(both):
    M, mesh, host, ora = both
    e = host.dump("TOPO_EDGES")
    assert np.array_equal(e[:, 0:2], ora.edge_nodes)
    assert np.array_equal(e[:, 2:4], ora.edge_elems)
    assert np.array_equal(e[:, 4:6], ora.edge_local)


def test_stencils_match_oracle_bit_exact(both):
    M, mesh, host, ora = both
    st = host.dump("TOPO_STENCILS")
    assert st.shape == ora.stencils.shape
    assert np.array_equal(st, ora.stencils)


def test_scheduling_stencils_match_oracle(both):
    M, mesh, host, ora = both
    ptr = host.dump("TOPO_SCHED_PTR")
    idx = host.dump("TOPO_SCHED_IDX")
    for i in range(mesh.n_elems):
        assert np.array_equal(idx[ptr[i]:ptr[i + 1]], ora.sched[i])


@pytest.mark.parametrize("M", [1, 2, 3])
def test_tables_match_oracle(M):
    mesh = strip_mesh(0, 1, 0, 1, 0.2, seed=1)
    host = HostTopology(mesh.nodes, mesh.tris, mesh.bedges, Config(M=M))
    nt = tb.nodal_tables(M)
    _, tm = tb.time_matrices(M)
    assert np.allclose(host.dump("TAB_DXI"), nt["Dxi"], atol=1e-12)
    assert np.allclose(host.dump("TAB_DETA"), nt["Deta"], atol=1e-12)
    assert np.allclose(host.dump("TAB_AMEAN"), nt["amean"], atol=1e-14)
    assert np.allclose(host.dump("TAB_EDGE"), nt["edge"], atol=1e-13)
    assert np.allclose(host.dump("TAB_AT"), tm["At"], atol=1e-13)
    assert np.allclose(host.dump("TAB_BT"), tm["Bt"], atol=1e-13)
    assert np.allclose(host.dump("TAB_DT"), tm["Dt"], atol=1e-12)
    g = host.dump("TAB_GAUSS")
    x, w = tb.gauss_legendre01(M + 1)
    assert np.allclose(g[0], x, atol=1e-15) and np.allclose(g[1], w, atol=1e-15)


@pytest.mark.parametrize("M", [1, 2, 3])
def test_modal_basis_gives_same_indicator(M):
    """The library's Dubiner basis and the oracle's Gram-Schmidt basis differ,
    but the oscillation indicator of a polynomial is basis independent."""
    mesh = strip_mesh(0, 1, 0, 1, 0.2, seed=1)
    host = HostTopology(mesh.nodes, mesh.tris, mesh.bedges, Config(M=M))
    C = host.dump("TAB_PSIC")        # psi_l = sum_k C[l,k] mono_k
    S = host.dump("TAB_SIGMA")
    rng = np.random.default_rng(M)
    xi, eta, w = tb.duffy_rule(M + 3)
    P_host = tb.eval_monomials(M, xi, eta) @ C.T
    P_ora = tb.eval_psi(M, xi, eta)
    assert np.allclose(P_host[:, 0], 1.0)
    gram = np.einsum("pl,pm,p->lm", P_host, P_host, w) / w.sum()
    assert np.abs(gram - np.eye(C.shape[0])).max() < 1e-12
    for _ in range(3):
        f = rng.normal(size=P_host.shape[1])
        vals = P_ora @ f
        ch = np.linalg.lstsq(P_host, vals, rcond=None)[0]
        assert abs(ch @ S @ ch - f @ tb.sigma_matrix(M) @ f) < 1e-10 * (1 + abs(f @ tb.sigma_matrix(M) @ f))


def test_degenerate_meshes_rejected():
    """Two triangles cannot fill a central stencil of n_e elements (the method
    needs them, eq. stencil): E_MESH, as the oracle refuses them; no element
    at all is an argument error."""
    nodes = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float)
    tris = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    be = np.array([[0, 1, 1], [1, 2, 1], [2, 3, 1], [3, 0, 1]], np.int32)
    for M in (1, 2, 3):
        with pytest.raises(_lib.AderError, match="E_MESH"):
            HostTopology(nodes, tris, be, Config(M=M))
        with pytest.raises(ValueError, match="too small"):
            build_topology(nodes, tris, M, be)
    with pytest.raises(_lib.AderError, match="E_ARG"):
        HostTopology(np.zeros((0, 2)), np.zeros((0, 3), np.int32), None, Config(M=1))


def test_transposed_stencil_rows():
    """The adjoint's gather lists: every row c >= 1 of every kept stencil
    appears exactly once, under the element it names, in ascending order."""
    mesh = square_graded_mesh(0.3, seed=3)
    for M in (1, 2):
        host = HostTopology(mesh.nodes, mesh.tris, mesh.bedges, Config(M=M))
        sten = host.dump("TOPO_STENCILS")             # (NE, 7, ne)
        NE, _, ne = sten.shape
        expect = {}
        for i in range(NE):
            for s in range(7):
                if sten[i, s, 0] < 0:
                    continue
                for c in range(1, ne):
                    expect.setdefault(int(sten[i, s, c]), []).append((i * ne + c) * 8 + s)
        ptr = host.dump("TOPO_TSTEN_PTR")
        idx = host.dump("TOPO_TSTEN_IDX")
        assert ptr[0] == 0 and ptr[-1] == idx.size
        for j in range(NE):
            got = idx[ptr[j]:ptr[j + 1]].tolist()
            assert got == sorted(expect.get(j, [])), j


def test_static_scratch_size_matches_the_header():
    import re
    from paper_1408_3719_amd import _lib
    hdr = open(os.path.join(ROOT, "include", "aderweno.h")).read()
    m = re.search(r"#define ADER_STATIC_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.STATIC_SCRATCH_BYTES
