"""The per-edge and per-row pieces of the moving-mesh adjoint
(paper_1408_3719_amd/csrc/lagadj.h) on the host: the space-time patch flux
(Rusanov and HLL) on interior, transmissive and slip-wall edges, also with
its corners at different times as in a cycle of the local time stepping, the
least-squares row geometry, the triangle area, and the Rusanov and HLL fluxes
(both upwind cases and the averaged one) through an unnormalised normal; each
vector-Jacobian product against central differences of its own forward
function at a seeded point, and the least-squares row against the monomial
means by a dense quadrature (tests/lagadj_fd.cpp, built with g++; no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1408_3719_amd", "csrc")

BOUND = {"patch_interior": 1e-8, "patch_transmissive": 1e-8, "patch_slip": 1e-8,
         "patch_hll_interior": 1e-8, "patch_hll_transmissive": 1e-8, "patch_hll_slip": 1e-8,
         "hll_middle": 1e-7, "hll_upwind_left": 1e-7, "hll_upwind_right": 1e-7, "ls_row": 1e-8,
         "ls_row_means": 1e-13, "area": 1e-8, "rusanov": 1e-7,
         "patch_lts_interior": 1e-8, "patch_lts_transmissive": 1e-8, "patch_lts_slip": 1e-8,
         "patch_lts_hll_interior": 1e-8, "patch_lts_hll_transmissive": 1e-8, "patch_lts_hll_slip": 1e-8}


@pytest.fixture(scope="module")
def lines(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = tmp_path_factory.mktemp("lagadj") / "lagadj_fd"
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    subprocess.run([gxx, "-std=c++17", "-O2", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(ROOT, "tests", "lagadj_fd.cpp"),
                    os.path.join(CSRC, "tables.cpp"), "-o", str(exe)], check=True, capture_output=True, timeout=300)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=120).stdout
    return [ln.split() for ln in out.strip().splitlines()]


def test_every_piece_and_order_is_checked(lines):
    seen = {(p, m) for p, m, _ in lines}
    for piece in ("patch_interior", "patch_transmissive", "patch_slip", "patch_hll_interior",
                  "patch_hll_transmissive", "patch_hll_slip", "patch_lts_interior", "patch_lts_transmissive",
                  "patch_lts_slip", "patch_lts_hll_interior", "patch_lts_hll_transmissive", "patch_lts_hll_slip",
                  "ls_row", "ls_row_means"):
        for M in (1, 2, 3):
            assert (piece, f"M={M}") in seen
    assert ("area", "M=0") in seen and ("rusanov", "M=0") in seen
    for piece in ("hll_middle", "hll_upwind_left", "hll_upwind_right"):
        assert (piece, "M=0") in seen


def test_products_match_central_differences(lines):
    for piece, m, dev in lines:
        assert float(dev) < BOUND[piece], (piece, m, dev)
