"""The benchmark's command-line contract that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_traffic_key_ignores_comments(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    d = bench.kernel_source_digest()
    assert len(d) == 64
    assert d == bench.kernel_source_digest()
