"""Host-side pieces of the benchmark contract (no GPU): the refusal of more
than one GPU and the arithmetic of the reported rates."""
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


def test_rate_arithmetic():
    """achieved = work per unit x units per launch / average launch time."""
    r = bench.rate_entry(25_000, 2_000_000, 40.0, 20, 78.6, 1e12)
    # 100k units per launch, 2 ms per launch: 2.5e9 flop / 2e-3 s = 1.25 TFLOP/s
    assert abs(r["achieved"] - 1.25) < 1e-12
    assert abs(r["frac"] - 1.25 / 78.6) < 1e-15
    assert r["units_per_launch"] == 100_000 and abs(r["avg_launch_us"] - 2000.0) < 1e-9
    h = bench.rate_entry(784, 1_000_000, 10.0, 10, 8000.0, 1e9)
    assert abs(h["achieved"] - 784 * 100_000 / 1e-3 / 1e9) < 1e-9


def test_unit_work_grows_with_the_order():
    for key, per in bench.UNIT_WORK.items():
        assert per[1] <= per[2] <= per[3], key
    # the kernels' own operation counts are of the same size as the method's
    for M in (1, 2, 3):
        assert 0.5 < bench.recon_flops(M) / bench.UNIT_WORK["recon_flops"][M] < 2.0
        assert 0.5 < bench.predict_flops(M) / bench.UNIT_WORK["predict_flops"][M] < 2.0


def test_traffic_table_covers_the_autotuner_candidates():
    assert set(bench.MEASURED_TRAFFIC["k_reconstruct"]) == set(bench.TRAFFIC_SWEEP)
    assert set(bench.MEASURED_TRAFFIC["k_predict"]) == set(bench.TRAFFIC_SWEEP)
