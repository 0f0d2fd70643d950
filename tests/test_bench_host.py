"""Host-side checks of bench.py (no GPU): the multi-GPU refusal, and that
the committed traffic summary under profiles/ belongs to the current
kernel sources and workload (else the bench would report traffic null)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_summary_matches_sources_and_workload():
    b = _bench()
    t = b.measured_traffic(65536, 15578)
    assert t is not None and t > 8.6e9         # at least the algorithmic bytes
    assert b.measured_traffic(65536, 15579) is None
    assert b.measured_traffic(1024, 15578) is None
