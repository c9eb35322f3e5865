"""Host-side checks of the benchmark script (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_figure_follows_the_pass_sources():
    sys.path.insert(0, ROOT)
    import bench
    t = bench.measured_traffic()
    # the committed counter summary either matches the pass sources (bytes of
    # one launch, above the 67.7 MB a plain pass must move) or is ignored
    assert t is None or 60_000_000 < t < 200_000_000
