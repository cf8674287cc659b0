"""bench.py's command-line contract that holds without a GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    for cfg in ("ba1m", "batch256", "grad100k", "rmat23", "trap", "group", "strata", "fastchol"):
        out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--config", cfg],
                             capture_output=True, text=True, timeout=120)
        assert out.returncode == 2
        assert "one GPU only" in out.stderr
        assert out.stdout == ""


def test_walk_bytes_counts_the_algorithmic_traffic():
    sys.path.insert(0, ROOT)
    import bench
    # 28 B per unweighted step, 16 B per attached and 8 B per scanned node per tree
    assert bench.walk_bytes(100, 2, 10, False) == 28 * 100 + 2 * (16 * 9 + 8 * 10)
    assert bench.walk_bytes(100, 2, 10, True) == 36 * 100 + 2 * (16 * 9 + 8 * 10)
