"""Host-side pieces of the benchmark contract (no GPU): the refusal of more
than one GPU, and the algorithmic operation counts the roofline uses (the
figures quoted in the design notes)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
    assert out.stdout.strip() == ""


def test_operation_counts():
    assert bench.recon_flops(2) == 29289
    assert bench.recon_flops(1) < bench.recon_flops(2) < bench.recon_flops(3)
    assert bench.predict_flops(1) < bench.predict_flops(2) < bench.predict_flops(3)
    assert bench.patch_bytes(2) == 760


def test_traffic_table_covers_the_autotuner_candidates():
    assert set(bench.MEASURED_TRAFFIC["k_reconstruct"]) == set(bench.TRAFFIC_SWEEP)
    assert set(bench.MEASURED_TRAFFIC["k_predict"]) == set(bench.TRAFFIC_SWEEP)
