"""The adjoint entry point that allocates nothing (ader_adjoint_gts_step_static,
scratch in the library's fixed device array) against ader_adjoint_gts_step
with a caller buffer, through the C ABI: two calls in a row, the second on a
smaller mesh, then a mesh too large for the fixed array."""
import ctypes

import numpy as np
import pytest

from workloads import explosion_case, vortex_case

pytestmark = pytest.mark.gpu


def _solver(mesh, Q0, M):
    from paper_1408_3719_amd import Config, Solver
    return Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=M, levels=1, mesh_velocity="eulerian"))


def _reference(s, dt, q, qb):
    """ader_adjoint_gts_step with a caller scratch filled with NaN bytes, so a
    read of anything the call did not write first would show in the result."""
    import torch
    n = ctypes.c_size_t()
    assert s.lib.ader_adjoint_workspace_size(s.ctx, ctypes.byref(n)) == 0
    buf = torch.full((n.value + 256,), 255, dtype=torch.uint8, device="cuda")
    aligned = (buf.data_ptr() + 255) // 256 * 256
    out = torch.full_like(qb, float("nan"))
    rc = s.lib.ader_adjoint_gts_step(s.ctx, dt, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(qb.data_ptr()),
                                     ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(aligned), n.value)
    assert rc == 0, s.lib.ader_last_error(s.ctx)
    torch.cuda.synchronize()
    return out, n.value


def _static(s, dt, q, qb):
    import torch
    out = torch.full_like(qb, float("nan"))
    rc = s.lib.ader_adjoint_gts_step_static(s.ctx, dt, ctypes.c_void_p(q.data_ptr()),
                                            ctypes.c_void_p(qb.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    assert rc == 0, s.lib.ader_last_error(s.ctx)
    torch.cuda.synchronize()
    return out


def test_static_adjoint_matches_the_caller_buffer_entry_point():
    import torch
    from paper_1408_3719_amd import _lib
    rng = np.random.default_rng(31)
    cases = [("explosion 6k, M=2", lambda: explosion_case(6000, seed=7), 2),
             ("vortex 900, M=2", lambda: vortex_case(900, seed=5), 2)]
    sizes = []
    for name, make, M in cases:
        mesh, Q0 = make()
        print(f"static adjoint: {name}, {mesh.n_elems} triangles", flush=True)
        s = _solver(mesh, Q0, M)
        dt = 0.5 * float(s.dump("DTCFL").min())
        Q = Q0 * (1.0 + 1e-3 * rng.standard_normal(Q0.shape))
        q = torch.tensor(Q.T.copy(), device="cuda")
        qb = torch.tensor(rng.standard_normal((4, mesh.n_elems)), device="cuda")
        ref, nbytes = _reference(s, dt, q, qb)
        got = _static(s, dt, q, qb)
        assert nbytes <= _lib.STATIC_SCRATCH_BYTES
        sizes.append(nbytes)
        r = ref.cpu().numpy()
        g = got.cpu().numpy()
        assert np.isfinite(r).all() and np.isfinite(g).all()
        # same kernels on the same inputs: identical to the last bit (and so
        # within the 1e-10 relative bar per variable)
        assert np.array_equal(g, r), np.abs(g - r).max()
        s.close()
    assert sizes[1] < sizes[0]                  # the second call was the smaller one


def test_static_adjoint_rejects_a_mesh_beyond_the_fixed_scratch():
    import torch
    from paper_1408_3719_amd import _lib
    mesh, Q0 = vortex_case(16_000, seed=2)
    s = _solver(mesh, Q0, 3)
    n = ctypes.c_size_t()
    assert s.lib.ader_adjoint_workspace_size(s.ctx, ctypes.byref(n)) == 0
    assert n.value > _lib.STATIC_SCRATCH_BYTES
    q = torch.tensor(Q0.T.copy(), device="cuda")
    out = torch.zeros_like(q)
    rc = s.lib.ader_adjoint_gts_step_static(s.ctx, 1e-4, ctypes.c_void_p(q.data_ptr()),
                                            ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(out.data_ptr()))
    assert rc == _lib.E_ARG
    assert "too large for the fixed adjoint scratch" in s.lib.ader_last_error(s.ctx).decode()
    torch.cuda.synchronize()
    assert not out.any()                        # nothing was launched
    s.close()
