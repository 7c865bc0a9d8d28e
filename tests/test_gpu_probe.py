"""The derivative-contraction measurement (ader_probe_contraction): the matrix
core variant (v_mfma_f64_16x16x4f64 over ten elements per wavefront) and the
vector variant compute the same rounds q <- q/2 + (D_xi q + D_eta q)/20 as a
NumPy evaluation with the library's own D_xi, D_eta (M = 2), element by
element, including a ragged last wavefront and idle lanes."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _solver():
    from paper_1408_3719_amd import Config, Solver
    from workloads import vortex_case
    mesh, Q0 = vortex_case(400, seed=5)
    return Solver(mesh.nodes, mesh.tris, mesh.bedges, Q0, Config(M=2, levels=1))


@pytest.mark.parametrize("n", [1, 37, 1013])
def test_probe_variants_match_numpy(n):
    import torch
    g = _solver()
    Dx, De = g.dump("TAB_DXI"), g.dump("TAB_DETA")
    rng = np.random.default_rng(n)
    F = rng.standard_normal((n, 10, 6))
    q = F.copy()
    for _ in range(5):
        d = np.einsum("km,efm->efk", Dx + De, q)
        q = 0.5 * q + 0.05 * d
    for mfma in (False, True):
        out, ms = g.probe_contraction(torch.tensor(F, device="cuda"), 5, mfma)
        got = out.cpu().numpy()
        print(f"n={n} mfma={mfma}: {ms:.3f} ms", flush=True)
        assert np.abs(got - q).max() <= 1e-13 * np.abs(q).max(), (mfma, np.abs(got - q).max())


def test_probe_rejects_bad_arguments():
    import torch
    from paper_1408_3719_amd import AderError
    g = _solver()
    with pytest.raises(AderError):
        g.probe_contraction(torch.zeros((4, 10, 6), device="cuda", dtype=torch.float64), 0, True)
    with pytest.raises(ValueError):
        g.probe_contraction(torch.zeros((4, 10, 5), device="cuda", dtype=torch.float64), 1, True)
