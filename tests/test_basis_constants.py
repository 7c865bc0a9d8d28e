"""The compile-time constants of the reference element used by the HIP
kernels (paper_1408_3719_amd/csrc/basis.h) against the oracle's own
definitions: the time Lagrange basis on the nodes q/M and its integrals, the
means of the monomials on the reference triangle, the oscillation-indicator
matrix (eq. Sigma) of the shifted monomials mapped to the oracle's
orthonormal basis, and the shifted monomials at the nodal lattice. A small
host program prints the constants (built with hipcc; no GPU is used)."""
import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from oracle import tables as tb  # noqa: E402

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

PROGRAM = r'''
#include <cstdio>
#include "basis.h"
using namespace aw;
template <int M> void dump(bool last) {
  constexpr int T = M + 1, nb = (M + 1) * (M + 2) / 2, nu = nb - 1;
  std::printf("\"%d\": {\"lag\": [", M);
  for (int q = 0; q < T; ++q)
    for (int k = 0; k < T; ++k) std::printf("%s%.17g", q + k ? ", " : "", TimePoly<M>::c.lag[q][k]);
  std::printf("], \"lint\": [");
  for (int q = 0; q < T; ++q)
    for (int k = 0; k <= T; ++k) std::printf("%s%.17g", q + k ? ", " : "", TimePoly<M>::c.lint[q][k]);
  std::printf("], \"mref\": [");
  for (int k = 0; k < nb; ++k) std::printf("%s%.17g", k ? ", " : "", RefMeans<M>::m[k]);
  std::printf("], \"sig\": [");
  for (int l = 0; l < nu; ++l)
    for (int m = 0; m < nu; ++m) std::printf("%s%.17g", l + m ? ", " : "", MonoBasis<M>::c.sig[l][m]);
  std::printf("], \"node\": [");
  for (int n = 0; n < nb; ++n)
    for (int l = 0; l < nu; ++l) std::printf("%s%.17g", n + l ? ", " : "", MonoBasis<M>::c.node[n][l]);
  std::printf("]}%s", last ? "" : ", ");
}
int main() {
  std::printf("{");
  dump<1>(false);
  dump<2>(false);
  dump<3>(true);
  std::printf("}\n");
  return 0;
}
'''


@pytest.fixture(scope="module")
def consts(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("basis")
    src, exe = d / "dump.hip", d / "dump"
    src.write_text(PROGRAM)
    inc = os.path.join(ROOT, "paper_1408_3719_amd", "csrc")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-std=c++17", "-O1", "-I", inc,
                    str(src), "-o", str(exe)], check=True, capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60)
    return {int(k): {n: np.array(v) for n, v in d.items()} for k, d in json.loads(out.stdout).items()}


@pytest.mark.parametrize("M", [1, 2, 3])
def test_time_basis_and_integrals(consts, M):
    T = M + 1
    lag = consts[M]["lag"].reshape(T, T)
    lint = consts[M]["lint"].reshape(T, T + 1)
    tau = np.linspace(-0.3, 1.3, 17)
    got = np.stack([np.polyval(lag[q][::-1], tau) for q in range(T)], -1)
    assert np.abs(got - tb.lagrange_time(M, tau)).max() < 1e-13
    got_i = np.stack([np.polyval(lint[q][::-1], tau) for q in range(T)], -1)
    ref_i = tb.lagrange_time_integral(M, np.zeros_like(tau), tau)
    assert np.abs(got_i - ref_i).max() < 1e-13


@pytest.mark.parametrize("M", [1, 2, 3])
def test_monomial_means_indicator_and_nodes(consts, M):
    mono = tb.monomials(M)
    nb = len(mono)
    nu = nb - 1
    mref = np.array([2.0 * float(tb.int_Te(a, b)) for a, b in mono])
    assert np.abs(consts[M]["mref"] - mref).max() < 1e-16
    # indicator: psi_l = sum_k C[l,k] mono_k with psi_l mean-free for l >= 1, so in
    # the shifted monomials Sigma_psi = C' S C'^T with C' = C[1:, 1:]
    S = consts[M]["sig"].reshape(nu, nu)
    C = tb.psi_coeffs(M)[1:, 1:]
    ref = tb.sigma_matrix(M)[1:, 1:]
    assert np.abs(C @ S @ C.T - ref).max() < 1e-13 * np.abs(ref).max()
    node = consts[M]["node"].reshape(nb, nu)
    xy = tb.nodal_xy(M)
    for n, (x, y) in enumerate(xy):
        exp = [x ** a * y ** b - mref[k] for k, (a, b) in enumerate(mono) if k > 0]
        assert np.abs(node[n] - exp).max() < 1e-15
