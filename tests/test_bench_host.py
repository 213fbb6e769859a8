"""Host-side checks of bench.py's contract (no GPU): one GPU only, and the
recorded sweep counters read back as integers or None."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == "" or not r.stdout.lstrip().startswith("{")


def test_recorded_counters_are_integers_or_none():
    import bench
    for key in ("traffic_bytes_per_launch", "valu_insts_per_launch"):
        v = bench.recorded_traffic(key)
        assert v is None or (isinstance(v, int) and v > 0)
    assert bench.recorded_traffic("no_such_figure") is None
